// Element-wise and reduction kernels of the CTMRG step (everything that is
// not a matrix product or the QR).
#pragma once
#include "common.hpp"

namespace ctm {

// out = sym(raw) / ||sym(raw)||_F; norm2_out[0] = ||sym(raw)||^2 (device).
void launch_symmetrize(hipStream_t s, const double* raw, double* out, int d, int D,
                       double* norm2_out);
// dev[0] = ||A - sym(A)||_F^2, dev[1] = ||A||_F^2.
void launch_symmetry_defect(hipStream_t s, const double* A, int d, int D, double* dev);
// a[(u,u'),(v,v'),(w,w')] = sum_s A[s,u,v,w] A[s,u',v',w'].
void launch_double_layer(hipStream_t s, const double* A, int d, int D, double* a);
// Double layer with physical legs open, stored [X][Y][Z][s][s'] (X, Y, Z
// fused ket/bra indices): rot = 0 -> A[s,x,y,z] A[s',x',y',z'];
// rot = 1 -> A[s,z,x,y] A[s',z',x',y'] (legs cycled).
void launch_double_layer_open(hipStream_t s, const double* A, int d, int D, int rot, double* aO);
// C = [[1]], T[0][(u,u')][0] = delta_{u u'}.
void launch_init_env(hipStream_t s, int D, double* C, double* T);
// dst[i] = (T)src[i].
// dst[r][c] = src[r][c] for a rows x cols FP64 block (row strides lds, ldd).
void launch_copy_block(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd,
                       int rows, int cols);
void launch_cast(hipStream_t s, const double* src, void* dst, DType t, int64_t n);
// dst (cols x rows, leading dimension rows) = (T) transpose of src (rows x
// cols, leading dimension cols).
void launch_cast_transpose(hipStream_t s, const double* src, void* dst, DType t, int rows,
                           int cols);
// Q = first k columns of the n x n identity, in type t, leading dimension ld.
void launch_eye(hipStream_t s, void* Q, DType t, int n, int k, int64_t ld);
// sgn[j] = -1 if M[j][j] < 0 else +1.
void launch_diag_signs(hipStream_t s, const double* M, int ld, int k, double* sgn);
// Q[:, j] *= sgn[j]; copy (nullable) = Q afterwards.
void launch_apply_signs(hipStream_t s, double* Q, int n, int k, const double* sgn, double* copy);
// Cout = sym(Cin) / ||sym(Cin)||_F (k x k); flag |= 1 if the norm is 0 or not finite.
// parts: at least CORNER_PARTS doubles of scratch for the partial sums.
constexpr int CORNER_PARTS = 256;
void launch_corner_finalize(hipStream_t s, const double* Cin, double* Cout, int k, double* parts,
                            int* flag);
// out = in / sqrt(sum of nparts partial sums of squares); flag as above.
void launch_scale_by_norm(hipStream_t s, const double* in, double* out, int64_t n,
                          const double* parts, int nparts, int* flag);
// M = M / max|M| (k x k).
void launch_scale_by_maxabs(hipStream_t s, double* M, int k);
// rho[(s,t),(s',t')] = R[s*d+s'][t*d+t'] / trace; out[0] = Tr(rho h), out[1..] = rho;
// flag |= 1 if the trace is 0 or not finite.
void launch_energy_finalize(hipStream_t s, const double* R, const double* h, int d, double* out,
                            int* flag);

}  // namespace ctm
