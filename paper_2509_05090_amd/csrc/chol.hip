// Cholesky factorization G = R^T R of a small symmetric matrix by one
// workgroup of 1024 threads (16 wavefronts): the lower triangle L = R^T is
// held packed in LDS and factored right-looking, one column per step (scale
// the column below its pivot, then update the trailing triangle), two
// barriers per column.  The first attempt runs on G itself; a pivot that is
// not positive, or below 64 u times its diagonal entry, restarts the
// factorization on G + s I with the shift of shifted Cholesky QR (Fukaya,
// Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 42
// (2020)), s = 11 (m k + k (k + 1)) u ||M||_F^2 with ||M||_F^2 = trace(G);
// a pivot that fails on the shifted matrix is clamped and reported.
#include "chol.hpp"

namespace ctm {

namespace {

constexpr int CT = 1024;
constexpr int CPACK = CHOL_KMAX * (CHOL_KMAX + 1) / 2;

__device__ __forceinline__ int pidx(int i, int j) { return (i * (i + 1)) / 2 + j; }  // j <= i

__global__ __launch_bounds__(CT) void cholesky_kernel(const double* __restrict__ G, int ldg, int k,
                                                      int m, double* __restrict__ R, int ldr,
                                                      int* __restrict__ status,
                                                      int* __restrict__ flag) {
  __shared__ double L[CPACK];
  __shared__ double col[CHOL_KMAX];    // the current column below its pivot, scaled
  __shared__ double rdiag[CHOL_KMAX];  // the pivots' square roots
  __shared__ double dref[CHOL_KMAX];   // diagonal of the matrix being factored
  __shared__ double wsum[CT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tx = tid & 31, ty = tid >> 5;
  const double u = 0x1p-53;

  // the shift from trace(G)
  double tr = 0.0;
  for (int i = tid; i < k; i += CT) tr += G[(int64_t)i * ldg + i];
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
  if (lane == 0) wsum[wv] = tr;
  __syncthreads();
  double trace = 0.0;
  for (int w = 0; w < CT / 64; ++w) trace += wsum[w];
  const double shift = 11.0 * ((double)m * k + (double)k * (k + 1)) * u * trace;

  int st = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double sh = attempt == 0 ? 0.0 : shift;
    for (int i = ty; i < k; i += 32) {
      const double* __restrict__ g = G + (int64_t)i * ldg;
      double* __restrict__ Lrow = &L[pidx(i, 0)];
      for (int j = tx; j <= i; j += 32) Lrow[j] = j == i ? g[j] + sh : g[j];
    }
    for (int i = tid; i < k; i += CT) dref[i] = G[(int64_t)i * ldg + i] + sh;
    __syncthreads();
    bool failed = false;  // uniform: every thread tests the same pivot
    for (int j = 0; j < k; ++j) {
      double d = L[pidx(j, j)];
      const double lim = 64.0 * u * dref[j];
      if (!(d > lim) || !(d <= 1.7e308)) {
        if (attempt == 0) {
          failed = true;
          break;
        }
        st |= 2;
        d = lim > 0.0 && lim <= 1.7e308 ? lim : 1.0;
      }
      const double r = sqrt(d), ri = 1.0 / r;
      if (tid == 0) rdiag[j] = r;
      for (int i = j + 1 + tid; i < k; i += CT) {
        const double v = L[pidx(i, j)] * ri;
        L[pidx(i, j)] = v;
        col[i] = v;
      }
      __syncthreads();
      for (int i = j + 1 + ty; i < k; i += 32) {
        const double li = col[i];
        double* __restrict__ Lrow = &L[pidx(i, 0)];
        for (int c = j + 1 + tx; c <= i; c += 32) Lrow[c] -= li * col[c];
      }
      __syncthreads();
    }
    if (!failed) break;
    st |= 1;
    __syncthreads();
  }

  // R = L^T: row i of R holds column i of L
  for (int i = ty; i < k; i += 32) {
    double* __restrict__ r = R + (int64_t)i * ldr;
    for (int j = tx; j < k; j += 32) r[j] = j > i ? L[pidx(j, i)] : (j == i ? rdiag[i] : 0.0);
  }
  if (tid == 0) {
    status[0] = st;
    if ((st & 2) && flag) atomicOr(flag, 2);
  }
}

}  // namespace

void launch_cholesky(hipStream_t s, const double* G, int ldg, int k, int m, double* R, int ldr,
                     int* status, int* flag) {
  if (k < 1 || k > CHOL_KMAX) throw std::invalid_argument("launch_cholesky: order out of range");
  cholesky_kernel<<<1, CT, 0, s>>>(G, ldg, k, m, R, ldr, status, flag);
  CTM_LAUNCHED();
}

}  // namespace ctm
