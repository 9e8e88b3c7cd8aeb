// Cholesky factorization G = R^T R of a small symmetric matrix and the
// inverse of its factor, blocked by 16, in one workgroup of four wavefronts.
//
// The lower block triangle of L = R^T sits in LDS as 16 x 16 blocks (rows
// padded to 17 doubles).  For block column J: wavefront 0 factors the
// diagonal block (unblocked, column by column, in registers with lane
// shuffles) and inverts it; then every wavefront takes blocks of the panel,
// L_IJ = A_IJ L_JJ^{-T}, and of the trailing update, A_IK -= L_IJ L_KJ^T,
// each a 16 x 16 x 16 product on the FP64 matrix cores (v_mfma_f64_16x16x4,
// four per block).  The inverse X = L^{-1} follows block row by block row:
// X_IJ = -L_II^{-1} sum_{K=J..I-1} L_IK X_KJ, overwriting row I of L once the
// row's sums are formed.  Only the 16-column diagonal factorizations are
// serial; everything else is matrix-core work with three (factorization) or
// two (inverse) barriers per block.  Orders that are not multiples of 16 are
// padded with an identity block.
//
// The first attempt factors G itself; a pivot that is not positive, or below
// 64 u times its diagonal entry, restarts the factorization on G + s I with
// the shift of shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa, Yamamoto,
// Yanagisawa, SIAM J. Sci. Comput. 42 (2020)), s = 11 (m k + k (k + 1)) u
// ||M||_F^2 with ||M||_F^2 = trace(G); a pivot that fails on the shifted
// matrix is clamped and reported.
#include "chol.hpp"

namespace ctm {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int CT = 256;
constexpr int CB = 16;                     // block order
constexpr int LDB = 17;                    // padded row length of a block in LDS
constexpr int BSZ = CB * LDB;              // doubles per block
constexpr int NBMAX = CHOL_KMAX / CB;      // blocks per dimension
constexpr int NBLK = NBMAX * (NBMAX + 1) / 2;
static_assert(NBMAX == 9 && CT == 256, "the inverse's work split assumes 9 block rows, 4 wavefronts");

__device__ __forceinline__ int bidx(int I, int J) { return (I * (I + 1)) / 2 + J; }  // J <= I

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / sqrt(d) for d > 0: the hardware estimate refined by two Newton steps
// inside a safe exponent range, else the library square root.
__device__ __forceinline__ double rsqrt_refined(double d) {
  if (!(d >= 0x1p-960 && d <= 0x1p960)) return 1.0 / sqrt(d);
  double y = __builtin_amdgcn_rsq(d);
  double e = fma(-d * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-d * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// acc += sgn * P Q^T for 16 x 16 blocks P, Q (rows of both read from LDS).
__device__ __forceinline__ d4v mma_abt(const double* P, const double* Q, double sgn, d4v acc,
                                       int r16, int grp) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sgn * P[r16 * LDB + 4 * s + grp],
                                               Q[r16 * LDB + 4 * s + grp], acc, 0, 0, 0);
  return acc;
}

// acc += sgn * P Q for 16 x 16 blocks P (rows read) and Q (columns read).
__device__ __forceinline__ d4v mma_ab(const double* P, const double* Q, double sgn, d4v acc,
                                      int r16, int grp) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sgn * P[r16 * LDB + 4 * s + grp],
                                               Q[(4 * s + grp) * LDB + r16], acc, 0, 0, 0);
  return acc;
}

// The MFMA result layout: lane (grp, r16), register r holds row 4 r + grp,
// column r16.
__device__ __forceinline__ d4v load_d(const double* B, int r16, int grp) {
  return d4v{B[grp * LDB + r16], B[(4 + grp) * LDB + r16], B[(8 + grp) * LDB + r16],
             B[(12 + grp) * LDB + r16]};
}
__device__ __forceinline__ void store_d(double* B, d4v v, int r16, int grp) {
#pragma unroll
  for (int r = 0; r < 4; ++r) B[(4 * r + grp) * LDB + r16] = v[r];
}

__global__ __launch_bounds__(CT) void cholesky_kernel(const double* __restrict__ G, int ldg, int k,
                                                      int m, double* __restrict__ R, int ldr,
                                                      double* __restrict__ Rinv, int ldi,
                                                      int* __restrict__ status,
                                                      int* __restrict__ flag) {
  __shared__ double A[NBLK * BSZ];      // L (then X) by blocks of the lower block triangle
  __shared__ double Dinv[NBMAX * BSZ];  // inverses of the diagonal blocks
  __shared__ double S[NBMAX * BSZ];     // block sums of the inverse's current row
  __shared__ double dref[NBMAX * CB];   // diagonal of the matrix being factored
  __shared__ double wsum[CT / 64];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, grp = lane >> 4;
  const int nb = (k + CB - 1) / CB, kp = nb * CB;
  const double u = 0x1p-53;

  double tr = 0.0;
  for (int i = tid; i < k; i += CT) tr += G[(int64_t)i * ldg + i];
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
  if (lane == 0) wsum[wv] = tr;
  __syncthreads();
  double trace = 0.0;
#pragma unroll
  for (int w = 0; w < CT / 64; ++w) trace += wsum[w];
  const double shift = 11.0 * ((double)m * k + (double)k * (k + 1)) * u * trace;

  int st = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double sh = attempt == 0 ? 0.0 : shift;
    // the lower block triangle of G (+ sh I), identity beyond k; one block
    // per pass, one entry per thread
    for (int I = 0; I < nb; ++I)
      for (int J = 0; J <= I; ++J) {
        const int i = CB * I + (tid >> 4), c = CB * J + (tid & 15);
        double v = i == c ? 1.0 : 0.0;
        if (i < k && c < k) v = G[(int64_t)i * ldg + c] + (i == c ? sh : 0.0);
        A[bidx(I, J) * BSZ + (tid >> 4) * LDB + (tid & 15)] = v;
      }
    for (int i = tid; i < kp; i += CT) dref[i] = i < k ? G[(int64_t)i * ldg + i] + sh : 1.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int J = 0; J < nb; ++J) {
      double* D = A + bidx(J, J) * BSZ;
      double* Di = Dinv + J * BSZ;
      if (wv == 0) {
        // diagonal block in registers, right-looking, one column per step:
        // lane (q, i) holds row i at columns 4 q .. 4 q + 3; the pivot is
        // read from its lane and the column's multipliers are broadcast
        // with lane shuffles, so a column costs no LDS round trip
        const int i = r16, q = grp;
        double a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = D[i * LDB + 4 * q + r];
        double rinv[CB];
        bool broke = false;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int jq = j >> 2, jr = j & 3;
          double d = __shfl(a[jr], CB * jq + j);
          const double lim = 64.0 * u * dref[J * CB + j];
          // multipliers of column j before scaling: A[i][j] for this row and
          // A[c][j] for this lane's columns c = 4 q + r
          const double li_raw = __shfl(a[jr], CB * jq + i);
          double lc_raw[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) lc_raw[r] = __shfl(a[jr], CB * jq + 4 * q + r);
          // the pivot test, wavefront-uniform; after a breakdown of the
          // unshifted attempt the remaining columns are skipped (no early
          // exit, so that the loop unrolls and a[], rinv[] stay in registers)
          const bool fail = !__builtin_amdgcn_readfirstlane((int)(d > lim && d <= 1.7e308));
          if (fail && attempt == 0) broke = true;
          if (!broke) {
            if (fail) {
              st |= 2;
              d = lim > 0.0 && lim <= 1.7e308 ? lim : 1.0;
            }
            const double ri = rsqrt_refined(d);
            rinv[j] = ri;
            const double lij = li_raw * ri;
            if (q == jq && i >= j) a[jr] = i == j ? d * ri : lij;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int c = 4 * q + r;
              if (c > j && c <= i) a[r] = fma(-lij, lc_raw[r] * ri, a[r]);
            }
          }
        }
        if (broke && lane == 0) bad = 1;
        if (!broke) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (4 * q + r <= i) D[i * LDB + 4 * q + r] = a[r];
        }
        wave_sync();  // the factor is in LDS before the inverse reads it
        // inverse of the diagonal block, column r16 by forward substitution
        // with the pivots' reciprocals (lanes 0..15); zeros above its diagonal
        if (lane < CB && !broke) {
          const int c = lane;
          double x[CB];
#pragma unroll
          for (int r = 0; r < CB; ++r) {
            double s0 = r == c ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int mm = 0; mm < r; ++mm) {
              const double t = D[r * LDB + mm] * (mm >= c ? x[mm] : 0.0);
              if (mm & 1) s1 -= t;
              else s0 -= t;
            }
            x[r] = r >= c ? (s0 + s1) * rinv[r] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < CB; ++r) Di[r * LDB + c] = x[r];
        }
      }
      __syncthreads();
      if (bad) break;  // uniform
      // panel: L_IJ = A_IJ Dinv^T
      for (int I = J + 1 + wv; I < nb; I += CT / 64) {
        double* B = A + bidx(I, J) * BSZ;
        const d4v v = mma_abt(B, Di, 1.0, d4v{0, 0, 0, 0}, r16, grp);
        wave_sync();  // the block's operand reads precede its overwrite
        store_d(B, v, r16, grp);
      }
      __syncthreads();
      // trailing update: A_IK -= L_IJ L_KJ^T for J < K <= I
      const int t = nb - J - 1, pairs = t * (t + 1) / 2;
      for (int p = wv; p < pairs; p += CT / 64) {
        int I = J + 1, rem = p;
        while (rem >= I - J) {  // p-th pair in row order: row I has I - J entries
          rem -= I - J;
          ++I;
        }
        const int K = J + 1 + rem;
        double* B = A + bidx(I, K) * BSZ;
        const d4v v = mma_abt(A + bidx(I, J) * BSZ, A + bidx(K, J) * BSZ, -1.0,
                              load_d(B, r16, grp), r16, grp);
        store_d(B, v, r16, grp);
      }
      __syncthreads();
    }
    if (!bad) break;
    st |= 1;
    __syncthreads();
  }

  // R = L^T, by 16 x 16 blocks of R: R[row][col] = L[col][row] for row <= col
  if (R) {
    for (int Ib = 0; Ib < nb; ++Ib)
#pragma unroll
      for (int Jb = 0; Jb < NBMAX; ++Jb) {
        const int rr = tid >> 4, cc = tid & 15, row = CB * Ib + rr, col = CB * Jb + cc;
        if (row < k && col < k)
          R[(int64_t)row * ldr + col] =
              (Jb > Ib || (Jb == Ib && cc >= rr)) ? A[bidx(Jb, Ib) * BSZ + cc * LDB + rr] : 0.0;
      }
  }
  if (Rinv) {
    // X = L^{-1} by block rows; X_II = Dinv[I]
    for (int I = 1; I < nb; ++I) {
      // block column J costs I - J products: wavefront w takes J = w and
      // J = 7 - w, which balances the chains (NBMAX = 9)
      for (int h = 0; h < 2; ++h) {
        const int J = h == 0 ? wv : NBMAX - 2 - wv;
        if (J >= I) continue;
        d4v acc{0, 0, 0, 0};
        for (int K = J; K < I; ++K)
          acc = mma_ab(A + bidx(I, K) * BSZ, K == J ? Dinv + J * BSZ : A + bidx(K, J) * BSZ, 1.0,
                       acc, r16, grp);
        store_d(S + J * BSZ, acc, r16, grp);
      }
      __syncthreads();
      for (int J = wv; J < I; J += CT / 64) {
        const d4v v = mma_ab(Dinv + I * BSZ, S + J * BSZ, -1.0, d4v{0, 0, 0, 0}, r16, grp);
        store_d(A + bidx(I, J) * BSZ, v, r16, grp);
      }
      __syncthreads();
    }
    // Rinv = X^T by blocks: Rinv[row][col] = X[col][row] for row <= col
    // (the block column loop unrolled, so that its LDS reads overlap)
    for (int Ib = 0; Ib < nb; ++Ib)
#pragma unroll
      for (int Jb = 0; Jb < NBMAX; ++Jb) {
        const int rr = tid >> 4, cc = tid & 15, row = CB * Ib + rr, col = CB * Jb + cc;
        if (row < k && col < k) {
          double v = 0.0;
          if (Jb > Ib) v = A[bidx(Jb, Ib) * BSZ + cc * LDB + rr];
          else if (Jb == Ib && cc >= rr) v = Dinv[Ib * BSZ + cc * LDB + rr];
          Rinv[(int64_t)row * ldi + col] = v;
        }
      }
  }
  if (tid == 0) {
    status[0] = st;
    if ((st & 2) && flag) atomicOr(flag, 2);
  }
}

}  // namespace

void launch_cholesky(hipStream_t s, const double* G, int ldg, int k, int m, double* R, int ldr,
                     double* Rinv, int ldi, int* status, int* flag) {
  if (k < 1 || k > CHOL_KMAX) throw std::invalid_argument("launch_cholesky: order out of range");
  cholesky_kernel<<<1, CT, 0, s>>>(G, ldg, k, m, R, ldr, Rinv, ldi, status, flag);
  CTM_LAUNCHED();
}

}  // namespace ctm
