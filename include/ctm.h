/*
 * ctm.h -- C interface of libctm: C3v-symmetric QR-based CTMRG for honeycomb
 * iPEPS on AMD Instinct MI355X (gfx950).
 *
 * Method: Q. Yang and P. Corboz, "Efficient iPEPS Simulation on the Honeycomb
 * Lattice via QR-based CTMRG", arXiv:2509.05090.
 *
 * Conventions shared by all calls
 *  - Site tensor A[s][u][v][w]: d x D x D x D, row-major FP64, real, projected
 *    onto the C3v-symmetric subspace of the trivial irrep (Appendix A:
 *    invariant under all permutations of the three virtual legs u, v, w).
 *  - Double layer a[I][J][K], I = u*D + u' (Sec. II.A, Fig. 1b).
 *  - Corner C[gamma][delta] (chi_c x chi_c), edge T[alpha][i][gamma]
 *    (chi_c x D^2 x chi_c; outer leg, end leg towards the apex, inner leg),
 *    projector P[(alpha,k)][mu] (chi_c D^2 x chi), all row-major FP64.
 *  - A local pair b[i][j][k][l] = sum_m a[i][j][m] a[m][k][l] is the four-leg
 *    tensor of the local mapping (Fig. 1c); one step enlarges the corner by a
 *    pair and two edges and renormalizes corner and edge with an isometry
 *    (Fig. 3a,b).
 *  - Device pointers are HIP device memory owned by the caller; `stream` is a
 *    hipStream_t (NULL = the default stream) on which all device work of a
 *    context is enqueued.  A call synchronizes the stream only when it returns
 *    values in host memory.
 *  - Every call returns CTM_OK (0) or a negative status; ctm_last_error()
 *    gives the reason.  After CTM_EDEVICE the context is unusable and may only
 *    be freed.  A context is not thread-safe; separate contexts are
 *    independent.
 */
#ifndef CTM_H
#define CTM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CTM_OK = 0,
  CTM_EINVAL = -1,     /* bad size, enum value or null pointer */
  CTM_ENOTSYM = -2,    /* ||A - sym(A)||_F > 1e-12 ||A||_F */
  CTM_ENOMEM = -3,     /* device allocation failed */
  CTM_EDEVICE = -4,    /* HIP runtime error; context poisoned */
  CTM_ENOTCONV = -5,   /* tolerance not reached within max_steps (state stays valid) */
  CTM_ENONFINITE = -6, /* NaN/Inf or zero norm in C or T */
  CTM_ESTATE = -7      /* call not valid in the current state */
};

/* Projector of the CTMRG step (Sec. II.B).
 * CTM_PROJ_QR:  thin QR of the chi_c D^2 x chi reduced corner M = Ct P_prev
 *               (Fig. 3d), Q1 R = M; the isometry is Q = Q1 gs(Q1^T P_prev),
 *               gs(X) the Gram-Schmidt basis of X's columns (QR with positive
 *               diagonal), which ties the basis inside span(Q1) to P_prev
 *               (the paper fixes none).  One sweep of orthogonal iteration
 *               per step: at a fixed point Q spans a dominant eigenspace of
 *               the enlarged corner Ct.  The first projector of an n-row
 *               corner is gs(first n rows of G).
 * CTM_PROJ_EVD: eigenvectors of Ct of the chi largest |eigenvalues| (Fig. 3c),
 *               ordered by decreasing |eigenvalue|, then larger eigenvalue;
 *               column signs follow P_prev when it matches n, else each
 *               column's largest entry is positive.  FP64 Householder
 *               tridiagonalization on the GPU, the tridiagonal eigenpairs on
 *               the host (bisection, inverse iteration), back-transformation
 *               on the GPU; the baseline the QR projector replaces.  Needs
 *               chi*D^2 <= 8192; synchronizes once per step.
 * CTM_PROJ_QR_CHOL: the CTM_PROJ_QR rule with Q1 from three Cholesky QR
 *               passes (Gram matrix on the matrix cores, blocked Cholesky of
 *               the chi x chi Gram matrix and the inverse of its factor,
 *               Q1 <- Q1 R^{-1}; gs(X) as in CTM_PROJ_QR), the first on
 *               M^T M + s I when M^T M is numerically singular (shifted
 *               Cholesky QR, Fukaya et al., SIAM J. Sci. Comput. 42 (2020)).
 *               Q depends on Q1 only through span(M), so it agrees with
 *               CTM_PROJ_QR to rounding while cond(M) stays below about 1e15;
 *               a Gram matrix that breaks down even when shifted sets the
 *               non-finite flag (CTM_ENONFINITE).  Needs chi <= 144.
 *               On a stream other than the NULL stream, FP64 and FP32 update
 *               steps form Ct Q1 and V Q1 on a pair of CU-masked streams
 *               that the library creates once per device and shares among
 *               its contexts (16 CUs factor X, the rest multiply) and finish the
 *               renormalization with (Ct Q1) gs(X) and (V Q1) gs(X); on the
 *               NULL stream (which synchronizes with such streams) the steps
 *               run in sequence.  Same result to rounding either way. */
typedef enum { CTM_PROJ_QR = 0, CTM_PROJ_EVD = 1, CTM_PROJ_QR_CHOL = 2 } ctm_proj;

/* Arithmetic of the contractions.  The QR, the sign gauge, the
 * normalization of C and T and the energy are FP64 in every mode; the master
 * copies of C, T and P are FP64.  FP32 and BF16 run the contractions on FP32
 * and BF16 matrix cores with FP32 accumulation.  CTM_PREC_LADDER starts on
 * BF16; ctm_converge moves it to FP32 when the spectrum change falls below
 * 1e-4 (or stops improving) and to FP64 below 1e-9, and reports convergence
 * only on the FP64 rung; ctm_step runs the current rung. */
typedef enum {
  CTM_PREC_FP64 = 0,
  CTM_PREC_FP32 = 1,
  CTM_PREC_BF16 = 2,
  CTM_PREC_LADDER = 3
} ctm_prec;

typedef struct {
  int d;        /* physical dimension, >= 1 */
  int D;        /* virtual bond dimension, >= 1 */
  int chi;      /* environment bond dimension, >= 1 */
  int proj;     /* ctm_proj */
  int prec;     /* ctm_prec */
} ctm_config;

typedef struct ctm_ctx ctm_ctx;

/* Project a raw tensor onto the C3v-symmetric subspace (Appendix A, trivial
 * irrep: mean over the 6 permutations of the virtual legs) and normalize it
 * to unit Frobenius norm.  raw_dev and A_dev: d*D^3 FP64 device arrays (may
 * alias).  Errors: CTM_EINVAL, CTM_ENONFINITE (zero projection). */
int ctm_symmetrize(const double *raw_dev, double *A_dev, int d, int D, void *stream);

/* Create a context.  Copies A (d*D^3, must be C3v-symmetric, else
 * CTM_ENOTSYM) and G (chi*D^2 x chi seeded N(0,1) start matrix: the first
 * projector of an n-row reduced corner is the Gram-Schmidt basis of G's
 * first n rows).  Builds the double layer and the small start environment
 * C = [[1]], T[0][(u,u')][0] = delta_{u u'} (chi_c = 1), and allocates all
 * device memory the run needs.  Errors: CTM_EINVAL, CTM_ENOTSYM, CTM_ENOMEM,
 * CTM_EDEVICE. */
int ctm_init(ctm_ctx **out, const ctm_config *cfg, const double *A_dev, const double *G_dev,
             void *stream);

/* Run n_steps >= 0 CTMRG steps (Fig. 3a,b; Sec. II.B): enlarged corner
 * Ct[(alpha,k),(beta,l)] = sum T[alpha,i,gamma] C[gamma,delta] T[beta,j,delta]
 * a[i,j,m] a[m,k,l]; projector Q (identity while chi_c D^2 <= chi);
 * C' = Q^T Ct Q symmetrized and T' = Q^T (T b) Q, both Frobenius-normalized.
 * The basis of Q follows the previous projector (see CTM_PROJ_QR), so a
 * converged environment is stationary element by element.  Nothing is synchronized
 * unless delta_host is non-null; then it receives the change of the
 * normalized corner spectrum across the last step (INFINITY if undefined).
 * Errors: CTM_EINVAL, CTM_ENONFINITE, CTM_EDEVICE. */
int ctm_step(ctm_ctx *c, int n_steps, double *delta_host);

/* Iterate until the corner-spectrum change is below tol, checking every
 * n_check >= 1 steps, or until max_steps steps were run.  steps_host and
 * delta_host (nullable) receive the steps taken and the last change.
 * Returns CTM_ENOTCONV if tol was not reached (the state stays usable). */
int ctm_converge(ctm_ctx *c, double tol, int max_steps, int n_check, int *steps_host,
                 double *delta_host);

/* Bond energy from the current environment (Sec. II.C, Fig. 4b): the
 * enlarged corner with the physical legs of its apex pair open, traced
 * against the rest of the six-corner ring Env = Q (Q^T Ct Q)^5 Q^T, where Q
 * is the projector the run's rule gives for the current state (the state is
 * not changed).  h_host: d^2 x d^2 row-major operator on (outer site, inner
 * site) of the pair.  e_host receives Tr(rho h)/Tr(rho); rho_host (nullable,
 * d^2 x d^2) the unit-trace bond density matrix rho[(s,t),(s',t')].  FP64.
 * Errors: CTM_EINVAL, CTM_ENONFINITE, CTM_EDEVICE. */
int ctm_energy(ctm_ctx *c, const double *h_host, double *e_host, double *rho_host);

/* Energy gradient with respect to the site tensor (Sec. II.D: the energy
 * differentiated through the CTMRG environment; the one-step adjoint of the
 * corner and edge contractions, of the two QR factorizations and of the
 * normalizations is written out as matrix products, all in FP64).
 * Needs a truncated environment (chi_c = chi < chi D^2, after at least one
 * truncating step), else CTM_ESTATE.  h_host: the d^2 x d^2 operator as for
 * ctm_energy; E = Tr(rho h)/Tr(rho).
 *  mode = k > 0: runs k CTMRG steps from the current state, evaluates E on
 *    the result and differentiates through the k steps with the current
 *    state held fixed (the paper's tracked steps); (C_i, T_i, P_i) of every
 *    step are kept and the step's intermediates recomputed on the way back.
 *    The state of the context is not changed.
 *  mode = 0: fixed-point adjoint at the current state, which must be a
 *    stationary point of the iteration (converged with ctm_converge):
 *    dE/dA = dE/dA|_env + sum_j (dF/dA)^T (J^T)^j dE/d(env), J the step's
 *    Jacobian; terms are added until one changes the cotangent of the
 *    double layer by less than tol relative to its norm (CTM_ENOTCONV after
 *    max_iter terms; the gradient is still written).  CTM_ESTATE (nothing
 *    written) if one step changes the unit-norm corner by more than 1e-5:
 *    where the corner spectrum comes in +-lambda pairs, C keeps turning
 *    within their eigenspaces at convergence (T, P, the spectrum and the
 *    energy converge), so the state is no fixed point; use mode k > 0.
 * gradA_dev: d*D^3 FP64 device buffer, receives the projection of dE/dA onto
 * the C3v-symmetric subspace.  e_host (nullable): E.  iters_host (nullable):
 * adjoint steps taken.  Allocates its workspace (about nine (chi D^2)^2 FP64
 * arrays) at the first call.  Errors: CTM_EINVAL, CTM_ESTATE, CTM_ENOTCONV,
 * CTM_ENONFINITE, CTM_ENOMEM, CTM_EDEVICE. */
int ctm_grad(ctm_ctx *c, const double *h_host, int mode, double tol, int max_iter,
             double *gradA_dev, double *e_host, int *iters_host);

/* Normalized corner spectrum of the current state: |eigenvalues| of C in
 * decreasing order divided by the largest.  s_host must hold chi values;
 * n_host receives chi_c.  Synchronizes.  Errors: CTM_EINVAL, CTM_EDEVICE. */
int ctm_spectrum(ctm_ctx *c, double *s_host, int *n_host);

/* Current sizes: chi_c, steps run so far, and the rows of the stored
 * projector (0 before the first truncation).  Any pointer may be null. */
int ctm_query(const ctm_ctx *c, int *chi_c, int *steps, int *p_rows);

/* Copy the environment into caller device buffers (C: chi_c^2, T:
 * chi_c*D^2*chi_c, P: p_rows*chi, each nullable).  Enqueued on the stream. */
int ctm_get_env(ctm_ctx *c, double *C_dev, double *T_dev, double *P_dev);

/* Replace the environment by caller device data of corner dimension chi_c
 * (1 <= chi_c <= chi) and a projector of p_rows rows (0 = none; else
 * p_rows = chi_c*D^2 of the state that produced it, P_dev non-null).
 * Enqueued on the stream.  Errors: CTM_EINVAL. */
int ctm_set_env(ctm_ctx *c, int chi_c, const double *C_dev, const double *T_dev, int p_rows,
                const double *P_dev);

/* Replace the site tensor of a context, keeping its environment (C, T,
 * P_prev), its buffers and its step count (Sec. II.D, Sec. III.B: each
 * energy evaluation of the variational optimization continues from the
 * environment of the previous one).  A_dev: d*D^3 FP64 device array, same d
 * and D as at ctm_init, C3v-symmetric (as for ctm_init).  The double layer
 * (and the open double layers of the energy) are rebuilt; the spectrum
 * history of ctm_step / ctm_converge restarts.  A rejected tensor leaves the
 * context unchanged.  Errors: CTM_EINVAL, CTM_ENOTSYM, CTM_ENONFINITE,
 * CTM_EDEVICE. */
int ctm_update_tensor(ctm_ctx *c, const double *A_dev);

/* Switch the contraction arithmetic of an existing context (for a precision
 * ladder: low precision far from convergence, FP64 near it). */
int ctm_set_precision(ctm_ctx *c, int prec);

/* Stages of a step timed by ctm_profile_read(). */
enum {
  CTM_STAGE_CORNER = 0,    /* enlarged corner (Fig. 3a,c): products 1-4 */
  CTM_STAGE_PROJECTOR = 1, /* reduced corner M = Ct P_prev, QR, basis (Fig. 3d) */
  CTM_STAGE_RENORM_C = 2,  /* C' = Q^T Ct Q, symmetrize, normalize (Fig. 3a) */
  CTM_STAGE_RENORM_T = 3,  /* T' = Q^T (T b) Q, normalize (Fig. 3b) */
  CTM_STAGE_BIG_GEMM = 4,  /* the three (chi_c D^2) x chi x (chi_c D^2) matrix-core
                              products with untransposed operands inside stages 1-3,
                              M = Ct P_prev, Ct Q, V Q (kernel time only) */
  CTM_NSTAGES = 5
};

/* Start (enable = 1) or stop (0) recording HIP events around every stage
 * of ctm_step on the context's stream; starting resets the totals. */
int ctm_profile(ctm_ctx *c, int enable);

/* Totals since the last reset (synchronizes): ms_host[CTM_NSTAGES] elapsed
 * GPU time, launches_host[CTM_NSTAGES] timed intervals, flops_host[0] the
 * algorithmic flop count of the CTM_STAGE_BIG_GEMM kernels (2 M N K each).
 * Any pointer may be null. */
int ctm_profile_read(ctm_ctx *c, double *ms_host, int64_t *launches_host, double *flops_host);

/* Free a context and all its device memory (null is ignored). */
void ctm_free(ctm_ctx *c);

/* Text of the last error of c, or of the last failed ctm_init/
 * ctm_symmetrize when c is null.  Valid until the next call on c. */
const char *ctm_last_error(const ctm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* CTM_H */
