// Element-wise and reduction kernels of the CTMRG step.
#include "kernels.hpp"

namespace ctm {

namespace {

constexpr int BT = 1024;  // threads of the single-workgroup kernels

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Sum over the block (blockDim.x a multiple of 64); every thread gets it.
__device__ double block_sum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

__device__ double block_max(double v, double* sh) {
  v = wmax(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
  __syncthreads();
  return t;
}

// Mean of A[s, p(u,v,w)] over the six permutations p of the virtual legs.
__device__ inline double sym_entry(const double* A, int D, int idx) {
  const int D3 = D * D * D;
  const int s = idx / D3, r = idx % D3;
  const int u = r / (D * D), v = (r / D) % D, w = r % D;
  const double* As = A + (size_t)s * D3;
  auto at = [&](int x, int y, int z) { return As[(x * D + y) * D + z]; };
  return (at(u, v, w) + at(u, w, v) + at(v, u, w) + at(v, w, u) + at(w, u, v) + at(w, v, u)) /
         6.0;
}

constexpr int SYM_PER_THREAD = 16;

__global__ __launch_bounds__(BT) void symmetrize_kernel(const double* raw, double* out, int d,
                                                        int D, double* norm2_out) {
  __shared__ double sh[BT / 64];
  const int N = d * D * D * D;
  double val[SYM_PER_THREAD];
  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < SYM_PER_THREAD; ++i) {
    const int idx = threadIdx.x + i * BT;
    val[i] = idx < N ? sym_entry(raw, D, idx) : 0.0;
    ss += val[i] * val[i];
  }
  const double nrm2 = block_sum(ss, sh);  // also orders all reads before the writes
  const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
#pragma unroll
  for (int i = 0; i < SYM_PER_THREAD; ++i) {
    const int idx = threadIdx.x + i * BT;
    if (idx < N) out[idx] = val[i] * inv;
  }
  if (threadIdx.x == 0) norm2_out[0] = nrm2;
}

__global__ __launch_bounds__(BT) void symmetry_defect_kernel(const double* A, int d, int D,
                                                             double* dev) {
  __shared__ double sh[BT / 64];
  const int N = d * D * D * D;
  double def = 0.0, nrm = 0.0;
  for (int idx = threadIdx.x; idx < N; idx += BT) {
    const double x = A[idx], y = sym_entry(A, D, idx);
    def += (x - y) * (x - y);
    nrm += x * x;
  }
  def = block_sum(def, sh);
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) {
    dev[0] = def;
    dev[1] = nrm;
  }
}

__global__ void double_layer_kernel(const double* A, int d, int D, double* a) {
  const int D2 = D * D, D3 = D2 * D;
  const int64_t total = (int64_t)D2 * D2 * D2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(idx / (D2 * D2)), J = (int)((idx / D2) % D2), K = (int)(idx % D2);
    const int ket = ((I / D) * D + J / D) * D + K / D, bra = ((I % D) * D + J % D) * D + K % D;
    double t = 0.0;
    for (int s = 0; s < d; ++s) t += A[s * D3 + ket] * A[s * D3 + bra];
    a[idx] = t;
  }
}

__global__ void double_layer_open_kernel(const double* A, int d, int D, int rot, double* aO) {
  const int D2 = D * D, D3 = D2 * D;
  const int64_t total = (int64_t)D2 * D2 * D2 * d * d;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int sp = (int)(idx % d), s = (int)((idx / d) % d);
    const int64_t ijk = idx / (d * d);
    const int X = (int)(ijk / (D2 * D2)), Y = (int)((ijk / D2) % D2), Z = (int)(ijk % D2);
    const int I = rot ? Z : X, J = rot ? X : Y, K = rot ? Y : Z;
    const int ket = ((I / D) * D + J / D) * D + K / D, bra = ((I % D) * D + J % D) * D + K % D;
    aO[idx] = A[s * D3 + ket] * A[sp * D3 + bra];
  }
}

__global__ void init_env_kernel(int D, double* C, double* T) {
  const int i = threadIdx.x;
  if (i == 0) C[0] = 1.0;
  for (int x = i; x < D * D; x += blockDim.x) T[x] = (x / D == x % D) ? 1.0 : 0.0;
}

// dst[r][c] = src[r][c] for a rows x cols block (row strides lds, ldd).
__global__ void copy_block_kernel(const double* __restrict__ src, int64_t lds,
                                  double* __restrict__ dst, int64_t ldd, int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

template <typename T>
__global__ void cast_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = from_f64<T>(src[i]);
}

// dst (cols x rows, ld rows) = (T) src^T (src rows x cols, ld cols), through
// 32 x 32 LDS tiles so that both sides are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void cast_transpose_kernel(const double* __restrict__ src,
                                                            T* __restrict__ dst, int rows,
                                                            int cols) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = src[(int64_t)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) dst[(int64_t)c * rows + r] = from_f64<T>(tile[tx][ty + k]);
  }
}

template <typename T>
__global__ void eye_kernel(T* Q, int n, int k, int64_t ld) {
  const int64_t total = (int64_t)n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k, c = i % k;
    Q[r * ld + c] = from_f64<T>(r == c ? 1.0 : 0.0);
  }
}

__global__ void diag_signs_kernel(const double* M, int ld, int k, double* sgn) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x)
    sgn[j] = M[(size_t)j * ld + j] < 0.0 ? -1.0 : 1.0;
}

__global__ void apply_signs_kernel(double* Q, int n, int k, const double* sgn, double* copy) {
  const int64_t total = (int64_t)n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = Q[i] * sgn[i % k];
    Q[i] = v;
    if (copy) copy[i] = v;
  }
}

// Symmetrized corner (C + C^T)/2 and per-block sums of squares.
__global__ __launch_bounds__(256) void sym_sumsq_kernel(const double* __restrict__ Cin,
                                                       double* __restrict__ Cout, int k,
                                                       double* __restrict__ parts) {
  __shared__ double sh[4];
  const int64_t total = (int64_t)k * k;
  double ss = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k, c = i % k;
    const double v = 0.5 * (Cin[i] + Cin[c * k + r]);
    Cout[i] = v;
    ss += v * v;
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = ss;
}

// out = in / sqrt(sum of parts); every block sums the parts in the same
// order.  Flags a zero or non-finite norm.
__global__ __launch_bounds__(256) void scale_by_norm_kernel(const double* in, double* out,
                                                           int64_t n, const double* parts,
                                                           int nparts, int* flag) {
  __shared__ double sh[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) t += parts[i];
  const double nrm = sqrt(block_sum(t, sh));
  const bool bad = !(nrm > 0.0) || !isfinite(nrm);
  const double inv = bad ? 0.0 : 1.0 / nrm;
  if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i] * inv;
}

__global__ __launch_bounds__(BT) void scale_by_maxabs_kernel(double* M, int k) {
  __shared__ double sh[BT / 64];
  const int total = k * k;
  double m = 0.0;
  for (int i = threadIdx.x; i < total; i += BT) m = fmax(m, fabs(M[i]));
  m = block_max(m, sh);
  const double inv = m > 0.0 ? 1.0 / m : 1.0;
  for (int i = threadIdx.x; i < total; i += BT) M[i] *= inv;
}

__global__ void energy_finalize_kernel(const double* R, const double* h, int d, double* out,
                                       int* flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int d2 = d * d;
  auto rho = [&](int x, int y) {  // x = (s,t), y = (s',t'); R rows (s,s'), columns (t,t')
    const int s = x / d, t = x % d, sp = y / d, tp = y % d;
    return R[(s * d + sp) * d2 + (t * d + tp)];
  };
  double tr = 0.0;
  for (int x = 0; x < d2; ++x) tr += rho(x, x);
  const bool bad = !(fabs(tr) > 0.0) || !isfinite(tr);
  if (bad) atomicOr(flag, 1);
  const double inv = bad ? 0.0 : 1.0 / tr;
  double e = 0.0;
  for (int x = 0; x < d2; ++x)
    for (int y = 0; y < d2; ++y) {
      const double r = rho(x, y) * inv;
      out[1 + x * d2 + y] = r;
      e += r * h[y * d2 + x];
    }
  out[0] = e;
}

inline unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 8192) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, cdiv(n, threads)));
}

}  // namespace

void launch_symmetrize(hipStream_t s, const double* raw, double* out, int d, int D,
                       double* norm2_out) {
  if ((int64_t)d * D * D * D > (int64_t)SYM_PER_THREAD * BT)
    throw std::invalid_argument("symmetrize: d*D^3 too large");
  symmetrize_kernel<<<1, BT, 0, s>>>(raw, out, d, D, norm2_out);
  CTM_LAUNCHED();
}

void launch_symmetry_defect(hipStream_t s, const double* A, int d, int D, double* dev) {
  symmetry_defect_kernel<<<1, BT, 0, s>>>(A, d, D, dev);
  CTM_LAUNCHED();
}

void launch_double_layer(hipStream_t s, const double* A, int d, int D, double* a) {
  const int64_t n = (int64_t)D * D * D * D * D * D;
  double_layer_kernel<<<grid_for(n), 256, 0, s>>>(A, d, D, a);
  CTM_LAUNCHED();
}

void launch_double_layer_open(hipStream_t s, const double* A, int d, int D, int rot, double* aO) {
  const int64_t n = (int64_t)D * D * D * D * D * D * d * d;
  double_layer_open_kernel<<<grid_for(n), 256, 0, s>>>(A, d, D, rot, aO);
  CTM_LAUNCHED();
}

void launch_init_env(hipStream_t s, int D, double* C, double* T) {
  init_env_kernel<<<1, 256, 0, s>>>(D, C, T);
  CTM_LAUNCHED();
}

void launch_copy_block(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd,
                       int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return;
  copy_block_kernel<<<grid_for(n), 256, 0, s>>>(src, lds, dst, ldd, rows, cols);
  CTM_LAUNCHED();
}

void launch_cast(hipStream_t s, const double* src, void* dst, DType t, int64_t n) {
  if (n <= 0) return;
  switch (t) {
    case DType::F64:
      CTM_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      return;
    case DType::F32: cast_kernel<float><<<grid_for(n), 256, 0, s>>>(src, (float*)dst, n); break;
    case DType::BF16: cast_kernel<bf16><<<grid_for(n), 256, 0, s>>>(src, (bf16*)dst, n); break;
  }
  CTM_LAUNCHED();
}

void launch_cast_transpose(hipStream_t s, const double* src, void* dst, DType t, int rows,
                           int cols) {
  if (rows <= 0 || cols <= 0) return;
  const dim3 grid((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32));
  switch (t) {
    case DType::F64:
      cast_transpose_kernel<double><<<grid, 256, 0, s>>>(src, (double*)dst, rows, cols);
      break;
    case DType::F32:
      cast_transpose_kernel<float><<<grid, 256, 0, s>>>(src, (float*)dst, rows, cols);
      break;
    case DType::BF16:
      cast_transpose_kernel<bf16><<<grid, 256, 0, s>>>(src, (bf16*)dst, rows, cols);
      break;
  }
  CTM_LAUNCHED();
}

void launch_eye(hipStream_t s, void* Q, DType t, int n, int k, int64_t ld) {
  const int64_t total = (int64_t)n * k;
  switch (t) {
    case DType::F64: eye_kernel<double><<<grid_for(total), 256, 0, s>>>((double*)Q, n, k, ld); break;
    case DType::F32: eye_kernel<float><<<grid_for(total), 256, 0, s>>>((float*)Q, n, k, ld); break;
    case DType::BF16: eye_kernel<bf16><<<grid_for(total), 256, 0, s>>>((bf16*)Q, n, k, ld); break;
  }
  CTM_LAUNCHED();
}

void launch_diag_signs(hipStream_t s, const double* M, int ld, int k, double* sgn) {
  diag_signs_kernel<<<1, 256, 0, s>>>(M, ld, k, sgn);
  CTM_LAUNCHED();
}

void launch_apply_signs(hipStream_t s, double* Q, int n, int k, const double* sgn, double* copy) {
  apply_signs_kernel<<<grid_for((int64_t)n * k), 256, 0, s>>>(Q, n, k, sgn, copy);
  CTM_LAUNCHED();
}

void launch_corner_finalize(hipStream_t s, const double* Cin, double* Cout, int k, double* parts,
                            int* flag) {
  const int64_t total = (int64_t)k * k;
  const int blocks = (int)std::min<int64_t>(CORNER_PARTS, std::max<int64_t>(1, (total + 1023) / 1024));
  sym_sumsq_kernel<<<blocks, 256, 0, s>>>(Cin, Cout, k, parts);
  CTM_LAUNCHED();
  scale_by_norm_kernel<<<blocks, 256, 0, s>>>(Cout, Cout, total, parts, blocks, flag);
  CTM_LAUNCHED();
}

void launch_scale_by_norm(hipStream_t s, const double* in, double* out, int64_t n,
                          const double* parts, int nparts, int* flag) {
  scale_by_norm_kernel<<<grid_for(n, 256, 1024), 256, 0, s>>>(in, out, n, parts, nparts, flag);
  CTM_LAUNCHED();
}

void launch_scale_by_maxabs(hipStream_t s, double* M, int k) {
  scale_by_maxabs_kernel<<<1, BT, 0, s>>>(M, k);
  CTM_LAUNCHED();
}

void launch_energy_finalize(hipStream_t s, const double* R, const double* h, int d, double* out,
                            int* flag) {
  energy_finalize_kernel<<<1, 64, 0, s>>>(R, h, d, out, flag);
  CTM_LAUNCHED();
}

}  // namespace ctm
