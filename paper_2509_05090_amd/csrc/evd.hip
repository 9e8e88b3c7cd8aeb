// Householder tridiagonalization (FP64) of the symmetric enlarged corner with
// the orthogonal factor accumulated, for the eigendecomposition projector.
//
// For column k the reflector H = I - tau v v^T maps A[k+1:, k] onto a
// multiple of e_1 (LAPACK's dlarfg convention); with p = tau A v and
// w = p - (tau/2)(p^T v) v the two-sided update is A <- A - v w^T - w v^T,
// and Q <- Q H.  Two kernels per column: the first forms v (every workgroup
// recomputes it from row k, which equals column k by symmetry) and the row
// products p = tau A v, q = Q v; the second applies the rank-two update to
// the trailing block of A and the rank-one update to Q.  Both triangles of
// A are kept, so rows are read contiguously.
#include "evd.hpp"

#include <algorithm>
#include <cmath>

#include "spectrum.hpp"

namespace ctm {

namespace {

constexpr int ET = 256;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ double block_sum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

constexpr int KA_ROWS = 32;  // rows per workgroup of the product kernel
constexpr int KB_ROWS = 8;   // rows per workgroup of the update kernel

// Reflector of column k from row k of A; v (length m = n-k-1) in LDS.
__device__ void make_reflector(const double* __restrict__ A, int n, int k, double* vs, double* sh,
                               double& tau, double& beta) {
  const int m = n - k - 1;
  const double* row = A + (int64_t)k * n + k + 1;
  double ss = 0.0;
  for (int j = 1 + threadIdx.x; j < m; j += ET) ss += row[j] * row[j];
  const double sigma = block_sum(ss, sh);
  const double x0 = row[0];
  double scale;
  if (sigma == 0.0) {
    tau = 0.0;
    beta = x0;
    scale = 0.0;
  } else {
    const double nrm = sqrt(x0 * x0 + sigma);
    beta = x0 >= 0.0 ? -nrm : nrm;
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  for (int j = threadIdx.x; j < m; j += ET) vs[j] = j == 0 ? 1.0 : row[j] * scale;
  __syncthreads();
}

// p[i] = tau sum_j A[i][k+1+j] v_j (i > k), q[i] = sum_j Q[i][k+1+j] v_j.
__global__ __launch_bounds__(ET) void trid_products_kernel(const double* __restrict__ A,
                                                           const double* __restrict__ Q, int n,
                                                           int k, double* __restrict__ v,
                                                           double* __restrict__ p,
                                                           double* __restrict__ q,
                                                           double* __restrict__ d,
                                                           double* __restrict__ e,
                                                           double* __restrict__ scal) {
  extern __shared__ double vs[];
  __shared__ double sh[ET / 64];
  double tau, beta;
  make_reflector(A, n, k, vs, sh, tau, beta);
  const int m = n - k - 1;
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j < m; j += ET) v[j] = vs[j];
    if (threadIdx.x == 0) {
      d[k] = A[(int64_t)k * n + k];
      e[k] = beta;
      scal[0] = tau;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r0 = blockIdx.x * KA_ROWS;
  for (int rr = wid; rr < KA_ROWS; rr += ET / 64) {
    const int i = r0 + rr;
    if (i >= n) break;
    const double* qrow = Q + (int64_t)i * n + k + 1;
    const double* arow = A + (int64_t)i * n + k + 1;
    double tq = 0.0, ta = 0.0;
    const bool lower = i > k;
    for (int j = lane; j < m; j += 64) {
      tq += qrow[j] * vs[j];
      if (lower) ta += arow[j] * vs[j];
    }
    tq = wsum(tq);
    ta = wsum(ta);
    if (lane == 0) {
      q[i] = tq;
      if (lower) p[i] = tau * ta;
    }
  }
}

// A[i][k+1+j] -= v_i w_j + w_i v_j (i > k), Q[i][k+1+j] -= tau q_i v_j,
// w = p - (tau/2)(p^T v) v.
__global__ __launch_bounds__(ET) void trid_update_kernel(double* __restrict__ A,
                                                         double* __restrict__ Q, int n, int k,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ scal) {
  __shared__ double sh[ET / 64];
  __shared__ double rv[KB_ROWS], rw[KB_ROWS], rq[KB_ROWS];
  const int m = n - k - 1;
  const double tau = scal[0];
  double t = 0.0;
  for (int j = threadIdx.x; j < m; j += ET) t += p[k + 1 + j] * v[j];
  const double alpha = 0.5 * tau * block_sum(t, sh);
  const int r0 = blockIdx.x * KB_ROWS;
  if (threadIdx.x < KB_ROWS) {
    const int i = r0 + threadIdx.x;
    const bool lower = i > k && i < n;
    const double vi = lower ? v[i - k - 1] : 0.0;
    rv[threadIdx.x] = vi;
    rw[threadIdx.x] = lower ? p[i] - alpha * vi : 0.0;
    rq[threadIdx.x] = i < n ? q[i] : 0.0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += ET) {
    const double vj = v[j];
    const double wj = p[k + 1 + j] - alpha * vj;
#pragma unroll
    for (int rr = 0; rr < KB_ROWS; ++rr) {
      const int i = r0 + rr;
      if (i >= n) break;
      double* qa = Q + (int64_t)i * n + k + 1 + j;
      *qa -= tau * rq[rr] * vj;
      if (i > k) {
        double* aa = A + (int64_t)i * n + k + 1 + j;
        *aa -= rv[rr] * wj + rw[rr] * vj;
      }
    }
  }
}

__global__ void trid_tail_kernel(const double* A, int n, double* d, double* e) {
  if (threadIdx.x != 0) return;
  if (n >= 2) {
    d[n - 2] = A[(int64_t)(n - 2) * n + n - 2];
    e[n - 2] = A[(int64_t)(n - 1) * n + n - 2];
  }
  d[n - 1] = A[(int64_t)(n - 1) * n + n - 1];
}

__global__ void widen_eye_kernel(const void* src, int t, double* A, double* Q, int64_t total,
                                 int n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x;
    if (t == 0) x = ((const double*)src)[i];
    else if (t == 1) x = (double)((const float*)src)[i];
    else x = (double)(float)((const bf16*)src)[i];
    A[i] = x;
    Q[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
}

// sgn[j] = sign of column j's overlap with P (>= 0 -> +1), or of its entry
// of largest magnitude (lowest row on ties) when P is null.
__global__ __launch_bounds__(ET) void column_signs_kernel(const double* __restrict__ U, int ldu,
                                                          int n, const double* __restrict__ P,
                                                          int ldp, double* __restrict__ sgn) {
  __shared__ double sh[ET / 64];
  __shared__ double bv[ET];
  __shared__ int bi[ET];
  const int j = blockIdx.x;
  if (P) {
    double t = 0.0;
    for (int r = threadIdx.x; r < n; r += ET) t += P[(int64_t)r * ldp + j] * U[(int64_t)r * ldu + j];
    t = block_sum(t, sh);
    if (threadIdx.x == 0) sgn[j] = t < 0.0 ? -1.0 : 1.0;
    return;
  }
  double best = -1.0;
  int at = n;
  for (int r = threadIdx.x; r < n; r += ET) {
    const double a = fabs(U[(int64_t)r * ldu + j]);
    if (a > best) {
      best = a;
      at = r;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = at;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t2 = 1; t2 < ET; ++t2)
      if (bv[t2] > best || (bv[t2] == best && bi[t2] < at)) {
        best = bv[t2];
        at = bi[t2];
      }
    sgn[j] = U[(int64_t)at * ldu + j] < 0.0 ? -1.0 : 1.0;
  }
}

__global__ void scale_columns_kernel(double* U, int ldu, int n, int k, const double* sgn) {
  const int64_t total = (int64_t)n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k, c = i % k;
    U[r * ldu + c] *= sgn[c];
  }
}

inline unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, cdiv(n, threads)));
}

}  // namespace

size_t evd_work_bytes(int n, int k) {
  return ((size_t)2 * n * n + 6 * (size_t)n + 8 + (size_t)n * k + k) * sizeof(double) + 256;
}

EvdWork evd_work_carve(void* p, int n, int k) {
  EvdWork w;
  w.n = n;
  w.k = k;
  double* d = (double*)p;
  w.A = d;
  d += (int64_t)n * n;
  w.Q = d;
  d += (int64_t)n * n;
  w.v = d;
  d += n;
  w.p = d;
  d += n;
  w.q = d;
  d += n;
  w.d = d;
  d += n;
  w.e = d;
  d += 2 * n;
  w.scal = d;
  d += 8;
  w.Z = d;
  d += (int64_t)n * k;
  w.sgn = d;
  return w;
}

void tridiagonalize(hipStream_t s, const void* A_in, DType t, int n, EvdWork& w) {
  if (n > w.n) throw std::invalid_argument("tridiagonalize: workspace too small");
  if (n > 8192) throw std::invalid_argument("tridiagonalize: n > 8192");
  widen_eye_kernel<<<grid_for((int64_t)n * n), 256, 0, s>>>(A_in, (int)t, w.A, w.Q,
                                                           (int64_t)n * n, n);
  CTM_LAUNCHED();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    trid_products_kernel<<<(unsigned)cdiv(n, KA_ROWS), ET, (size_t)m * sizeof(double), s>>>(
        w.A, w.Q, n, k, w.v, w.p, w.q, w.d, w.e, w.scal);
    CTM_LAUNCHED();
    trid_update_kernel<<<(unsigned)cdiv(n, KB_ROWS), ET, 0, s>>>(w.A, w.Q, n, k, w.v, w.p, w.q,
                                                                 w.scal);
    CTM_LAUNCHED();
  }
  trid_tail_kernel<<<1, 64, 0, s>>>(w.A, n, w.d, w.e);
  CTM_LAUNCHED();
}

void eigh_top(hipStream_t s, const void* A_in, DType t, int n, int k, EvdWork& w, const Scratch& ws,
              double* U, int ldu, const double* P, std::vector<double>& lam_host) {
  if (k > w.k || k > n) throw std::invalid_argument("eigh_top: bad k");
  tridiagonalize(s, A_in, t, n, w);
  std::vector<double> d(n), e(std::max(n - 1, 0));
  CTM_HIP(hipMemcpyAsync(d.data(), w.d, n * sizeof(double), hipMemcpyDeviceToHost, s));
  if (n > 1)
    CTM_HIP(hipMemcpyAsync(e.data(), w.e, (n - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipStreamSynchronize(s));
  std::vector<double> z;
  tridiag_top_eigenpairs(d, e, k, lam_host, z);
  CTM_HIP(hipMemcpyAsync(w.Z, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice, s));
  // U = Q Z
  gemm(s, DType::F64, n, k, n, Operand{w.Q, n, false}, Operand{w.Z, k, false},
       Output{U, ldu, DType::F64}, 1, 1, 1.0, 0.0, ws);
  column_signs_kernel<<<k, ET, 0, s>>>(U, ldu, n, P, k, w.sgn);
  CTM_LAUNCHED();
  scale_columns_kernel<<<grid_for((int64_t)n * k), 256, 0, s>>>(U, ldu, n, k, w.sgn);
  CTM_LAUNCHED();
  CTM_HIP(hipStreamSynchronize(s));  // z is host memory read by the copy above
}

}  // namespace ctm
