// C entry points of the step's building blocks (see include/ctm_kernels.h).
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ctm.h"
#include "ctm_kernels.h"
#include "chol.hpp"
#include "gemm.hpp"
#include "qr.hpp"
#include "evd.hpp"

using namespace ctm;

namespace ctm {
void set_global_error(const std::string& s);
}

namespace {

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { CTM_HIP(hipMalloc(&p, bytes ? bytes : 8)); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

__global__ void copy_upper_kernel(const double* M, int ld, int k, double* R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * k) return;
  const int r = i / k, c = i % k;
  R[i] = c >= r ? M[(size_t)r * ld + c] : 0.0;
}

}  // namespace

extern "C" int ctm_gemm(int prec, int M, int N, int K, const void* A, int64_t lda, int transA,
                        int64_t sA0, int64_t sA1, const void* B, int64_t ldb, int transB,
                        int64_t sB0, int64_t sB1, void* C, int64_t ldc, int ctype, int64_t sC0,
                        int64_t sC1, int nb0, int nb1, double alpha, double beta, int ksplit,
                        void* stream) {
  if (prec < 0 || prec > 2 || ctype < 0 || ctype > 2 || M < 0 || N < 0 || K < 1 || nb0 < 1 ||
      nb1 < 1 || !A || !B || !C || ksplit < 0) {
    set_global_error("ctm_gemm: bad arguments");
    return CTM_EINVAL;
  }
  try {
    const DType e = (DType)prec;
    const size_t wsb = (ksplit > 1 || nb0 * nb1 == 1) ? gemm_scratch_bytes(e, M, N) : 0;
    DevBuf ws(wsb);
    gemm((hipStream_t)stream, e, M, N, K, Operand{A, lda, transA != 0, sA0, sA1},
         Operand{B, ldb, transB != 0, sB0, sB1}, Output{C, ldc, (DType)ctype, sC0, sC1}, nb0, nb1,
         alpha, beta, Scratch{ws.p, wsb}, ksplit);
    CTM_HIP(hipStreamSynchronize((hipStream_t)stream));
    return CTM_OK;
  } catch (const DeviceError& ex) {
    set_global_error(ex.what());
    return CTM_EDEVICE;
  } catch (const std::exception& ex) {
    set_global_error(ex.what());
    return CTM_EINVAL;
  }
}

extern "C" int ctm_qr(const double* M_dev, int n, int k, double* Q_dev, double* R_dev,
                      void* stream) {
  if (!M_dev || !Q_dev || k < 1 || n < k || n > QR_MAX_ROWS) {
    set_global_error("ctm_qr: bad arguments");
    return CTM_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf Mw((size_t)n * k * 8), ws(qr_work_bytes(n, k));
    QrWork w = qr_work_carve(s, ws.p, n, k);
    CTM_HIP(hipMemcpyAsync(Mw.p, M_dev, (size_t)n * k * 8, hipMemcpyDeviceToDevice, s));
    householder_qr(s, (double*)Mw.p, k, n, k, w);
    householder_form_q(s, w, n, k, Q_dev, k);
    if (R_dev) {
      copy_upper_kernel<<<(unsigned)cdiv((int64_t)k * k, 256), 256, 0, s>>>((const double*)Mw.p, k,
                                                                            k, R_dev);
      CTM_LAUNCHED();
    }
    CTM_HIP(hipStreamSynchronize(s));
    return CTM_OK;
  } catch (const DeviceError& ex) {
    set_global_error(ex.what());
    return CTM_EDEVICE;
  } catch (const std::exception& ex) {
    set_global_error(ex.what());
    return CTM_EINVAL;
  }
}

extern "C" int ctm_cholesky(const double* G_dev, int k, int m, double* R_dev, double* Rinv_dev,
                            int* status_host, void* stream) {
  if (!G_dev || !R_dev || !status_host || k < 1 || k > CHOL_KMAX || m < 1) {
    set_global_error("ctm_cholesky: bad arguments");
    return CTM_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf st(sizeof(int) * 4);
    launch_cholesky(s, G_dev, k, k, m, R_dev, k, Rinv_dev, k, (int*)st.p, nullptr);
    CTM_HIP(hipMemcpyAsync(status_host, st.p, sizeof(int), hipMemcpyDeviceToHost, s));
    CTM_HIP(hipStreamSynchronize(s));
    return CTM_OK;
  } catch (const DeviceError& ex) {
    set_global_error(ex.what());
    return CTM_EDEVICE;
  } catch (const std::exception& ex) {
    set_global_error(ex.what());
    return CTM_EINVAL;
  }
}

extern "C" int ctm_eigh(const double* A_dev, int n, int k, const double* P_dev, double* U_dev,
                        double* lam_host, void* stream) {
  if (!A_dev || !U_dev || !lam_host || n < 1 || k < 1 || k > n || n > 8192) {
    set_global_error("ctm_eigh: bad arguments");
    return CTM_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf w(evd_work_bytes(n, k)), ws(gemm_scratch_bytes(DType::F64, n, k));
    EvdWork ew = evd_work_carve(w.p, n, k);
    std::vector<double> lam;
    eigh_top(s, A_dev, DType::F64, n, k, ew, Scratch{ws.p, gemm_scratch_bytes(DType::F64, n, k)},
             U_dev, k, P_dev, lam);
    for (int i = 0; i < k; ++i) lam_host[i] = lam[i];
    return CTM_OK;
  } catch (const DeviceError& ex) {
    set_global_error(ex.what());
    return CTM_EDEVICE;
  } catch (const std::exception& ex) {
    set_global_error(ex.what());
    return CTM_EINVAL;
  }
}
