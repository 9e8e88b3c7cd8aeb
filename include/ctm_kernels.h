/*
 * ctm_kernels.h -- the building blocks of libctm's CTMRG step, exported so
 * that each can be checked on its own.
 *
 * Conventions as in ctm.h: device pointers are HIP device memory owned by
 * the caller, `stream` is a hipStream_t, calls return CTM_OK (0) or a
 * negative status (CTM_EINVAL for bad arguments, CTM_ENOMEM, CTM_EDEVICE),
 * and ctm_last_error(NULL) explains the last failure.
 */
#ifndef CTM_KERNELS_H
#define CTM_KERNELS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types of ctm_gemm operands: 0 = FP64, 1 = FP32, 2 = BF16. */

/* C = alpha * op(A) op(B) + beta * C on the matrix cores, for nb0 x nb1
 * batches.  op(A) is M x K: element (r, k) at A[r*lda + k], or A[k*lda + r]
 * if transA; op(B) is K x N: element (k, c) at B[k*ldb + c], or
 * B[c*ldb + k] if transB; C element (r, c) at C[r*ldc + c].  Batch (b0, b1)
 * offsets A, B and C by b0*s?0 + b1*s?1 elements.  A and B have element type
 * `prec` (FP64 accumulates in FP64, FP32 and BF16 in FP32); C has type
 * `ctype`, which must equal `prec` for batched products.  ksplit: 0 = choose,
 * 1 = no split of the k range, >1 = that many partial sums (unbatched only),
 * reduced in a fixed order.  Scratch is allocated per call. */
int ctm_gemm(int prec, int M, int N, int K,
             const void *A, int64_t lda, int transA, int64_t sA0, int64_t sA1,
             const void *B, int64_t ldb, int transB, int64_t sB0, int64_t sB1,
             void *C, int64_t ldc, int ctype, int64_t sC0, int64_t sC1,
             int nb0, int nb1, double alpha, double beta, int ksplit, void *stream);

/* Thin QR of the n x k FP64 matrix M (row-major, n >= k >= 1) by blocked
 * Householder reflections (Sec. II.B, Fig. 3d: the factorization behind the
 * projector).  Q_dev (n x k) receives the explicit orthonormal factor and
 * R_dev (k x k, nullable) the upper-triangular factor, with LAPACK's sign
 * convention R[j][j] = -sign(pivot) * ||column||.  M_dev is not modified. */
int ctm_qr(const double *M_dev, int n, int k, double *Q_dev, double *R_dev, void *stream);

/* Cholesky factorization G = R^T R of the symmetric k x k FP64 matrix G_dev
 * (row-major, lower triangle read; 1 <= k <= 144), taken as the Gram matrix
 * of an m x k matrix: the factor of the Cholesky QR projector
 * (CTM_PROJ_QR_CHOL), by one workgroup.  R_dev (k x k) receives the upper
 * triangle with a positive diagonal, zeros below; Rinv_dev (k x k, nullable)
 * receives R^{-1}, likewise upper triangular.  If a pivot is not
 * positive (or below 64 u times its diagonal entry) the factorization is
 * redone on G + s I, s = 11 (m k + k (k + 1)) u trace(G) (shifted Cholesky
 * QR, Fukaya et al., SIAM J. Sci. Comput. 42 (2020)), and bit 0 of
 * *status_host is set; bit 1 if the shifted matrix broke down too (pivots
 * clamped).  Synchronizes. */
int ctm_cholesky(const double *G_dev, int k, int m, double *R_dev, double *Rinv_dev,
                 int *status_host, void *stream);

/* Eigenvectors of the k eigenvalues of largest magnitude of the symmetric
 * n x n FP64 matrix A_dev (row-major, 1 <= k <= n <= 8192; the
 * eigendecomposition projector's solver, Sec. II.B, Fig. 3c).  U_dev (n x k)
 * receives them ordered by decreasing |eigenvalue|, then larger eigenvalue;
 * column signs: non-negative overlap with P_dev's columns (n x k, nullable),
 * else largest entry positive.  lam_host (k) receives the eigenvalues.
 * A_dev is not modified.  Synchronizes. */
int ctm_eigh(const double *A_dev, int n, int k, const double *P_dev, double *U_dev,
             double *lam_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTM_KERNELS_H */
