// Shared definitions of the CTMRG HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace ctm {

typedef __bf16 bf16;

// Element types of device buffers.
enum class DType : int { F64 = 0, F32 = 1, BF16 = 2 };

inline size_t dtype_size(DType t) {
  return t == DType::F64 ? 8 : (t == DType::F32 ? 4 : 2);
}

// A HIP runtime failure; carries the call site for the context's error text.
struct DeviceError : std::runtime_error {
  explicit DeviceError(const std::string& s) : std::runtime_error(s) {}
};

#define CTM_HIP(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::ctm::DeviceError(std::string(#call) + " failed: " +               \
                               hipGetErrorString(e_) + " (" + __FILE__ + ":" +   \
                               std::to_string(__LINE__) + ")");                  \
  } while (0)

#define CTM_LAUNCHED() CTM_HIP(hipGetLastError())

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T> __device__ inline T from_f64(double x);
template <> __device__ inline double from_f64<double>(double x) { return x; }
template <> __device__ inline float from_f64<float>(double x) { return (float)x; }
template <> __device__ inline bf16 from_f64<bf16>(double x) { return (bf16)(float)x; }

template <typename T> __device__ inline double to_f64(T x) { return (double)(float)x; }
template <> __device__ inline double to_f64<double>(double x) { return x; }
template <> __device__ inline double to_f64<float>(float x) { return (double)x; }

template <typename To, typename From> __device__ inline To convert(From x);
template <> __device__ inline double convert<double, double>(double x) { return x; }
template <> __device__ inline float convert<float, float>(float x) { return x; }
template <> __device__ inline bf16 convert<bf16, bf16>(bf16 x) { return x; }
template <> __device__ inline float convert<float, double>(double x) { return (float)x; }
template <> __device__ inline bf16 convert<bf16, double>(double x) { return (bf16)(float)x; }
template <> __device__ inline bf16 convert<bf16, float>(float x) { return (bf16)x; }
template <> __device__ inline double convert<double, float>(float x) { return (double)x; }
template <> __device__ inline float convert<float, bf16>(bf16 x) { return (float)x; }
template <> __device__ inline double convert<double, bf16>(bf16 x) { return (double)(float)x; }

}  // namespace ctm
