// Cholesky factorization of a small Gram matrix (FP64, one workgroup).
#pragma once
#include "common.hpp"

namespace ctm {

// Largest order the single-workgroup factorization holds in LDS (the lower
// block triangle of 16 x 16 blocks, the diagonal blocks' inverses and one
// block row of sums); a multiple of 16.
constexpr int CHOL_KMAX = 144;

// G = R^T R for the symmetric k x k matrix G (leading dimension ldg; only its
// lower triangle is read), R upper triangular with a positive diagonal,
// written to R (k x k, leading dimension ldr, zeros below the diagonal) and
// its inverse to Rinv (leading dimension ldi); either output nullable.
// G is taken as the Gram matrix M^T M of an m x k matrix M.  When a pivot is
// not positive (or below 64 u times its diagonal entry) the factorization
// restarts on G + s I with s = 11 (m k + k (k + 1)) u trace(G), the shift of
// shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
// SIAM J. Sci. Comput. 42 (2020)), and bit 0 of status[0] is set; if the
// shifted matrix breaks down too, the pivots are clamped, bit 1 of status[0]
// is set and flag[0] |= 2 (flag nullable).  k <= CHOL_KMAX.
void launch_cholesky(hipStream_t s, const double* G, int ldg, int k, int m, double* R, int ldr,
                     double* Rinv, int ldi, int* status, int* flag);

}  // namespace ctm
