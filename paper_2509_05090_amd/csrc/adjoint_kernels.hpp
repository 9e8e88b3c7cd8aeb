// Element-wise, permutation and reduction kernels of the CTMRG adjoint.
#pragma once
#include "common.hpp"

namespace ctm {

// out[a][c][b][d] = in[a][b][c][d] (dims A, B, C, Dd); out += if accumulate.
void launch_swap_mid(hipStream_t s, const double* in, double* out, int A, int B, int C, int Dd,
                     bool accumulate);
// out = copy of the lower triangle mirrored: out[i][j] = in[max(i,j)][min(i,j)] (k x k).
void launch_copyltu(hipStream_t s, const double* in, double* out, int k);
// out = R^{-1} diag(sgn) for the upper triangle of R (k x k, leading dimension ldr);
// sgn nullable (= all ones).  One thread per column, back substitution.
void launch_tri_inv_upper(hipStream_t s, const double* R, int ldr, int k, const double* sgn,
                          double* out);
// Deterministic dot product: out[0] = sum a[i] b[i] (two passes through `parts`,
// which holds DOT_PARTS doubles).
constexpr int DOT_PARTS = 256;
void launch_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* parts,
                double* out);
// out = (g - y * dot[0]) / nrm[0] (n elements): adjoint of y = x / ||x|| given
// dot = <y, g> and nrm = ||x||.
void launch_unit_norm_bwd(hipStream_t s, const double* g, const double* y, const double* dot,
                          const double* nrm, double* out, int64_t n);
// Forward of the corner finalization keeping its norm: S = (Cq + Cq^T)/2,
// nrm[0] = ||S||_F, Cn = S / nrm[0] (k x k, single workgroup).
void launch_corner_fwd(hipStream_t s, const double* Cq, double* Cn, double* nrm, int k);
// Adjoint of the corner finalization: out = sym((g - Cn <Cn, g>) / nrm).
void launch_corner_bwd(hipStream_t s, const double* g, const double* Cn, const double* nrm,
                       double* out, int k);
// sc[0] = max |M|, out = M / sc[0] (k x k).
void launch_maxabs_scale(hipStream_t s, const double* M, double* out, double* sc, int k);
// out = alpha (M + M^T) / sc[0] (k x k); sc nullable (= 1).
void launch_sym_scaled(hipStream_t s, const double* M, const double* sc, double alpha, double* out,
                       int k);
// out = M / sc[0] (n elements).
void launch_div_scalar(hipStream_t s, const double* M, const double* sc, double* out, int64_t n);
// Bond energy and its adjoint: R[(s,s')][(t,t')] (d^2 x d^2) -> e = Tr(rho h),
// rho(x,y) = R/tr with x = (s,t), y = (s',t'); Rb = d e / d R.  out[0] = e.
void launch_energy_bwd(hipStream_t s, const double* R, const double* h, int d, double* out,
                       double* Rb);
// out[i] = beta out[i] + sum_b in[b len + i].
void launch_sum_batches(hipStream_t s, const double* in, int nb, int64_t len, double* out,
                        double beta);
// gA += adjoint of a = sum_s A (x) A through the ket and bra factors.
void launch_double_layer_bwd(hipStream_t s, const double* ab, const double* A, int d, int D,
                             double* gA);
// gA += adjoint of the open double layer (rot as in launch_double_layer_open).
void launch_double_layer_open_bwd(hipStream_t s, const double* aOb, const double* A, int d, int D,
                                  int rot, double* gA);
// out = sym(g) (mean over the 6 virtual-leg permutations), no normalization.
void launch_symmetrize_plain(hipStream_t s, const double* g, double* out, int d, int D);
// out = in (n doubles).
void launch_copy(hipStream_t s, const double* in, double* out, int64_t n);
// p[i] = 0 (n doubles).
void launch_zero(hipStream_t s, double* p, int64_t n);
// y += alpha x (n doubles).
void launch_axpy(hipStream_t s, const double* x, double* y, int64_t n, double alpha);
// nrm[0] = sqrt(sumsq[0]); out = in / nrm[0] (n doubles).
void launch_normalize(hipStream_t s, const double* in, const double* sumsq, double* nrm, double* out,
                      int64_t n);

}  // namespace ctm
