// Energy gradient of the QR-based C3v CTMRG with respect to the site tensor
// (Sec. II.D: the paper differentiates through k tracked CTMRG steps).
//
// The forward step x = (C, T, P) -> x' = (C', T', Q) is recomputed in FP64
// with every intermediate kept (the "tape"), and its adjoint is written out
// by hand as matrix products of the same shapes as the forward ones:
//   corner/edge normalization  y = s / ||s||:  s_bar = (y_bar - y <y, y_bar>) / ||s||
//   C' = Q^T Ct Q, T' = Q^T V3, V3 <- V2 <- V = T (x) a: transposed products
//   Q = Q1 Qx, Qx Rx = X = Q1^T P (positive diagonal), Q1 R1 = M = Ct P:
//       the QR adjoint for a tall full-rank factorization (Walter and
//       Lehmann 2018; Liao, Liu, Wang, Xiang, PRX 9, 031041 (2019)):
//       A_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^{-T}
//   Ct = (T C T) (x) a (x) a: transposed products, index regroupings by the
//       swap kernels.
// Contributions to the cotangent of the double layer a may be stored with
// its legs permuted: a is built from A by the same leg permutations, so
// for a C3v-symmetric A the projection onto the symmetric subspace of the
// resulting dE/dA is unchanged.
//
// Modes: k > 0 runs k steps from the current state (checkpoints of
// (C_i, T_i, P_i), the tape recomputed on the way back), evaluates the
// energy and back-propagates, leaving the state unchanged; k = 0 treats the
// current state as the fixed point x* = F(x*) and sums the adjoint series
// x_bar <- J^T x_bar until a term adds less than tol (relative) to the
// double-layer cotangent.  (The environment cotangent itself need not decay
// to zero: gauge rotations of the kept basis are marginal directions of the
// step, and rounding leaves components along them that the energy does not
// see.)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint_kernels.hpp"
#include "context.hpp"
#include "kernels.hpp"

namespace ctm {

struct Tape {
  double *TCp, *V, *W, *Ct, *M, *Q1, *R1i, *X, *Xw, *Qx, *Rxi, *sgn, *Q, *Gm, *Cq, *Cn, *V2, *V3,
      *Tr, *Tn;
  double* sc;  // nS, nT, sumsq(T), max|Cq|
};

struct GradBuffers {
  Tape tp;
  double *bQ, *bV3, *bV2, *bV, *bCt, *bCtP, *bW, *bWP, *WP, *bTCp, *bTCpP, *TP, *bTP;
  double *bQx, *bQ1, *Mx, *Mxs, *Tmp, *bX, *M1, *M1s, *bM, *QC, *bCq, *bTr;
  double *ab, *abpart, *aOb, *aOrb, *gA;
  double *xC[2], *xT[2], *xP[2];
  double *Cr, *Cr2, *Cr4, *Cr5, *bCr, *bCr2, *bCr4, *bCr5, *QC5, *bQC5, *EnvP, *TCTp, *XO, *EO;
  double *R, *Rb, *bXO, *bEO, *TCpT, *bTCpT, *bTe, *h, *eout, *dots, *parts, *abprev;
  std::vector<double*> ckC, ckT, ckP;
};

void free_grad(GradBuffers* g) { delete g; }

namespace {

struct Dims {
  int x, D2, n, d, dd;
  int64_t D4, D6, NT;
};

Dims dims_of(const ctm_ctx* c) {
  Dims g;
  g.x = c->chi;
  g.D2 = c->D2;
  g.n = c->chi * c->D2;
  g.d = c->d;
  g.dd = c->d * c->d;
  g.D4 = (int64_t)g.D2 * g.D2;
  g.D6 = g.D4 * g.D2;
  g.NT = (int64_t)g.x * g.D2 * g.x;
  return g;
}

void mm(ctm_ctx* c, int M, int N, int K, const double* A, int64_t lda, bool ta, const double* B,
        int64_t ldb, bool tb, double* C, int64_t ldc, double alpha = 1.0, double beta = 0.0) {
  gemm(c->stream, DType::F64, M, N, K, Operand{A, lda, ta}, Operand{B, ldb, tb},
       Output{C, ldc, DType::F64}, 1, 1, alpha, beta, c->ws);
}

void ensure_grad_buffers(ctm_ctx* c) {
  if (c->grad) return;
  const Dims g = dims_of(c);
  const int64_t x = g.x, n = g.n, x2 = x * x, nn = (int64_t)n * n, nx = (int64_t)n * x;
  const int64_t xD2 = x2 * g.D2, xo = xD2 * g.dd;
  auto* b = new GradBuffers();
  c->grad = b;
  auto A = [&](int64_t cnt) { return c->allocd(std::max<int64_t>(cnt, 1)); };
  Tape& t = b->tp;
  t.TCp = A(x * n);
  t.V = A(nn);
  t.W = A(nx);
  t.Ct = A(nn);
  t.M = A(nx);
  t.Q1 = A(nx);
  t.R1i = A(x2);
  t.X = A(x2);
  t.Xw = A(x2);
  t.Qx = A(x2);
  t.Rxi = A(x2);
  t.sgn = A(x);
  t.Q = A(nx);
  t.Gm = A(nx);
  t.Cq = A(x2);
  t.Cn = A(x2);
  t.V2 = A(nx);
  t.V3 = A(nn);
  t.Tr = A(g.NT);
  t.Tn = A(g.NT);
  t.sc = A(8);
  b->bQ = A(nx);
  b->bV3 = A(nn);
  b->bV2 = A(nx);
  b->bV = A(nn);
  b->bCt = A(nn);
  b->bCtP = A(nn);
  b->bW = A(nx);
  b->bWP = A(xD2);
  b->WP = A(xD2);
  b->bTCp = A(x * n);
  b->bTCpP = A(x * n);
  b->TP = A(xD2);
  b->bTP = A(xD2);
  b->bQx = A(x2);
  b->bQ1 = A(nx);
  b->Mx = A(x2);
  b->Mxs = A(x2);
  b->Tmp = A(x2);
  b->bX = A(x2);
  b->M1 = A(x2);
  b->M1s = A(x2);
  b->bM = A(nx);
  b->QC = A(nx);
  b->bCq = A(x2);
  b->bTr = A(g.NT);
  b->ab = A(g.D6);
  b->abpart = A(x * g.D6);
  b->aOb = A(g.D6 * g.dd);
  b->aOrb = A(g.D6 * g.dd);
  b->gA = A((int64_t)g.d * c->D * c->D * c->D);
  for (int i = 0; i < 2; ++i) {
    b->xC[i] = A(x2);
    b->xT[i] = A(g.NT);
    b->xP[i] = A(nx);
  }
  b->Cr = A(x2);
  b->Cr2 = A(x2);
  b->Cr4 = A(x2);
  b->Cr5 = A(x2);
  b->bCr = A(x2);
  b->bCr2 = A(x2);
  b->bCr4 = A(x2);
  b->bCr5 = A(x2);
  b->QC5 = A(nx);
  b->bQC5 = A(nx);
  b->EnvP = A(nn);
  b->TCTp = A(nn);
  b->XO = A(xo);
  b->EO = A(xo);
  b->bXO = A(xo);
  b->bEO = A(xo);
  b->R = A((int64_t)g.dd * g.dd);
  b->Rb = A((int64_t)g.dd * g.dd);
  b->TCpT = A(x * n);
  b->bTCpT = A(x * n);
  b->bTe = A(nx);
  b->h = A((int64_t)g.dd * g.dd);
  b->eout = A(8);
  b->dots = A(8);
  b->parts = A(DOT_PARTS);
  b->abprev = A(g.D6);
}

// Forward step at (C, T, P) in FP64, keeping every intermediate (Sec. II.B,
// Fig. 3; the same schedule as the engine's step).
void tape_forward(ctm_ctx* c, const double* C, const double* T, const double* P) {
  const Dims g = dims_of(c);
  const int x = g.x, D2 = g.D2, n = g.n;
  hipStream_t s = c->stream;
  Tape& t = c->grad->tp;
  const double* a = c->a;
  const DType f = DType::F64;
  // TCp[beta][gamma][j] = sum_delta C[gamma][delta] T[beta][j][delta]
  gemm(s, f, x, D2, x, Operand{C, x, false}, Operand{T, x, true, (int64_t)D2 * x},
       Output{t.TCp, D2, f, (int64_t)x * D2}, x, 1, 1.0, 0.0, c->ws);
  // V[(alpha,m)][(gamma,j)] = sum_i T[alpha][i][gamma] a[m][i][j]
  gemm(s, f, x, D2, D2, Operand{T, x, true, (int64_t)D2 * x, 0},
       Operand{a, D2, false, 0, (int64_t)D2 * D2}, Output{t.V, D2, f, (int64_t)D2 * n, n}, x, D2,
       1.0, 0.0, c->ws);
  mm(c, n, x, n, t.V, n, false, t.TCp, n, true, t.W, x);  // W = V TCp^T
  // Ct[(alpha,k)][(beta,l)] = sum_m W[(alpha,m)][beta] a[m][k][l]
  gemm(s, f, x, D2, D2, Operand{t.W, x, true, (int64_t)D2 * x, 0},
       Operand{a, (int64_t)D2 * D2, false, 0, D2}, Output{t.Ct, D2, f, (int64_t)D2 * n, n}, x,
       D2, 1.0, 0.0, c->ws);
  // reduced corner and its QR: M = Ct P = Q1 R1
  mm(c, n, x, n, t.Ct, n, false, P, x, false, t.M, x);
  householder_qr(s, t.M, x, n, x, c->qr);
  householder_form_q(s, c->qr, n, x, t.Q1, x);
  launch_tri_inv_upper(s, t.M, x, x, nullptr, t.R1i);
  // basis tied to P: X = Q1^T P = Qx Rx (diag(Rx) > 0), Q = Q1 Qx
  mm(c, x, x, n, t.Q1, x, true, P, x, false, t.X, x);
  launch_copy(s, t.X, t.Xw, (int64_t)x * x);
  householder_qr(s, t.Xw, x, x, x, c->qr);
  householder_form_q(s, c->qr, x, x, t.Qx, x);
  launch_diag_signs(s, t.Xw, x, x, t.sgn);
  launch_apply_signs(s, t.Qx, x, x, t.sgn, nullptr);
  launch_tri_inv_upper(s, t.Xw, x, x, t.sgn, t.Rxi);
  mm(c, n, x, x, t.Q1, x, false, t.Qx, x, false, t.Q, x);
  // C' = sym(Q^T Ct Q) / ||.||
  mm(c, n, x, n, t.Ct, n, false, t.Q, x, false, t.Gm, x);
  mm(c, x, x, n, t.Q, x, true, t.Gm, x, false, t.Cq, x);
  launch_corner_fwd(s, t.Cq, t.Cn, t.sc + 0, x);
  // T' = Q^T V3 / ||.||, V3[alpha][(k,l)][nu] = sum_m a[k][l][m] (V Q)[(alpha,m)][nu]
  mm(c, n, x, n, t.V, n, false, t.Q, x, false, t.V2, x);
  gemm(s, f, D2 * D2, x, D2, Operand{a, D2, false, 0}, Operand{t.V2, x, false, (int64_t)D2 * x},
       Output{t.V3, x, f, (int64_t)D2 * D2 * x}, x, 1, 1.0, 0.0, c->ws);
  mm(c, x, D2 * x, n, t.Q, x, true, t.V3, (int64_t)D2 * x, false, t.Tr, (int64_t)D2 * x);
  launch_dot(s, t.Tr, t.Tr, g.NT, c->grad->parts, t.sc + 2);
  launch_normalize(s, t.Tr, t.sc + 2, t.sc + 1, t.Tn, g.NT);
}

// Adjoint of the projector (QR of M = Ct P and the basis tied to P): given
// bQ, accumulates into bCt and writes bP.
void proj_bwd(ctm_ctx* c, const double* P, double* bP) {
  const Dims g = dims_of(c);
  const int x = g.x, n = g.n;
  GradBuffers& b = *c->grad;
  const Tape& t = b.tp;
  hipStream_t s = c->stream;
  // Q = Q1 Qx
  mm(c, x, x, n, t.Q1, x, true, b.bQ, x, false, b.bQx, x);
  mm(c, n, x, x, b.bQ, x, false, t.Qx, x, true, b.bQ1, x);
  // Qx Rx = X: X_bar = (Qx_bar + Qx copyltu(-Qx_bar^T Qx)) Rx^{-T}
  mm(c, x, x, x, b.bQx, x, true, t.Qx, x, false, b.Mx, x, -1.0);
  launch_copyltu(s, b.Mx, b.Mxs, x);
  launch_copy(s, b.bQx, b.Tmp, (int64_t)x * x);
  mm(c, x, x, x, t.Qx, x, false, b.Mxs, x, false, b.Tmp, x, 1.0, 1.0);
  mm(c, x, x, x, b.Tmp, x, false, t.Rxi, x, true, b.bX, x);
  // X = Q1^T P
  mm(c, n, x, x, P, x, false, b.bX, x, true, b.bQ1, x, 1.0, 1.0);
  mm(c, n, x, x, t.Q1, x, false, b.bX, x, false, bP, x);
  // Q1 R1 = M: M_bar = (Q1_bar + Q1 copyltu(-Q1_bar^T Q1)) R1^{-T}
  mm(c, x, x, n, b.bQ1, x, true, t.Q1, x, false, b.M1, x, -1.0);
  launch_copyltu(s, b.M1, b.M1s, x);
  mm(c, n, x, x, t.Q1, x, false, b.M1s, x, false, b.bQ1, x, 1.0, 1.0);
  mm(c, n, x, x, b.bQ1, x, false, t.R1i, x, true, b.bM, x);
  // M = Ct P
  mm(c, n, n, x, b.bM, x, false, P, x, true, b.bCt, n, 1.0, 1.0);
  mm(c, n, x, n, t.Ct, n, false, b.bM, x, false, bP, x, 1.0, 1.0);
}

// Adjoint of Ct = W (x) a (first half): from bCt to bW, bV (+= if accV) and
// bTCp; accumulates into ab.
void ct_bwd_w(ctm_ctx* c, bool accV) {
  const Dims g = dims_of(c);
  const int x = g.x, D2 = g.D2, n = g.n;
  GradBuffers& b = *c->grad;
  const Tape& t = b.tp;
  hipStream_t s = c->stream;
  const double* a = c->a;
  const DType f = DType::F64;
  launch_swap_mid(s, b.bCt, b.bCtP, x, D2, x, D2, false);  // [a][k][b][l] -> [a][b][k][l]
  launch_swap_mid(s, t.W, b.WP, x, D2, x, 1, false);       // [a][m][b] -> [a][b][m]
  // bWP[(a,b)][m] = sum_(k,l) bCtP[(a,b)][(k,l)] a[m][(k,l)]
  gemm(s, f, x * x, D2, (int)g.D4, Operand{b.bCtP, g.D4, false}, Operand{a, g.D4, true},
       Output{b.bWP, D2, f}, 1, 1, 1.0, 0.0, c->ws);
  // ab[m][(k,l)] += sum_(a,b) WP[(a,b)][m] bCtP[(a,b)][(k,l)]
  gemm(s, f, D2, (int)g.D4, x * x, Operand{b.WP, D2, true}, Operand{b.bCtP, g.D4, false},
       Output{b.ab, g.D4, f}, 1, 1, 1.0, 1.0, c->ws);
  launch_swap_mid(s, b.bWP, b.bW, x, x, D2, 1, false);  // [a][b][m] -> [a][m][b]
  // W = V TCp^T
  mm(c, n, n, x, b.bW, x, false, t.TCp, n, false, b.bV, n, 1.0, accV ? 1.0 : 0.0);
  mm(c, x, n, n, b.bW, x, true, t.V, n, false, b.bTCp, n);
}

// Adjoint of V = T (x) a and TCp = C T (second half): from bV and bTCp to
// the cotangents of C and T (written to oC, oT); accumulates into ab.
void ct_bwd_v(ctm_ctx* c, const double* C, const double* T, double* oC, double* oT) {
  const Dims g = dims_of(c);
  const int x = g.x, D2 = g.D2, n = g.n;
  GradBuffers& b = *c->grad;
  hipStream_t s = c->stream;
  const double* a = c->a;
  const DType f = DType::F64;
  double* bVP = b.bCtP;
  launch_swap_mid(s, b.bV, bVP, x, D2, x, D2, false);  // [a][m][g][j] -> [a][g][m][j]
  launch_swap_mid(s, T, b.TP, x, D2, x, 1, false);     // T[a][i][g] -> TP[a][g][i]
  // bTP[(a,g)][i] = sum_(m,j) bVP[(a,g)][(m,j)] a[i][m][j]   (a symmetric in its legs)
  gemm(s, f, x * x, D2, (int)g.D4, Operand{bVP, g.D4, false}, Operand{a, g.D4, true},
       Output{b.bTP, D2, f}, 1, 1, 1.0, 0.0, c->ws);
  launch_swap_mid(s, b.bTP, oT, x, x, D2, 1, false);  // [a][g][i] -> [a][i][g]
  // ab (legs permuted) += TP^T bVP
  gemm(s, f, D2, (int)g.D4, x * x, Operand{b.TP, D2, true}, Operand{bVP, g.D4, false},
       Output{b.ab, g.D4, f}, 1, 1, 1.0, 1.0, c->ws);
  // TCp[b][g][j] = sum_d C[g][d] T[b][j][d]
  launch_swap_mid(s, b.bTCp, b.bTCpP, 1, x, x, D2, false);  // [b][g][j] -> [g][b][j]
  mm(c, x, x, n, b.bTCpP, n, false, T, x, false, oC, x);
  gemm(s, f, D2, x, x, Operand{b.bTCp, D2, true, (int64_t)x * D2}, Operand{C, x, false},
       Output{oT, x, f, (int64_t)D2 * x}, x, 1, 1.0, 1.0, c->ws);
}

// One-step adjoint at the tape's state: (iC, iT, iP) cotangents of
// (C', T', P') -> (oC, oT, oP) cotangents of (C, T, P); ab accumulates the
// double-layer part.
void step_vjp(ctm_ctx* c, const double* C, const double* T, const double* P, const double* iC,
              const double* iT, const double* iP, double* oC, double* oT, double* oP) {
  const Dims g = dims_of(c);
  const int x = g.x, D2 = g.D2, n = g.n;
  GradBuffers& b = *c->grad;
  const Tape& t = b.tp;
  hipStream_t s = c->stream;
  const double* a = c->a;
  const DType f = DType::F64;
  // normalizations
  launch_corner_bwd(s, iC, t.Cn, t.sc + 0, b.bCq, x);
  launch_dot(s, t.Tn, iT, g.NT, b.parts, b.dots + 0);
  launch_unit_norm_bwd(s, iT, t.Tn, b.dots + 0, t.sc + 1, b.bTr, g.NT);
  // T' = Q^T V3
  launch_copy(s, iP, b.bQ, (int64_t)n * x);
  mm(c, n, x, D2 * x, t.V3, (int64_t)D2 * x, false, b.bTr, (int64_t)D2 * x, true, b.bQ, x, 1.0,
     1.0);
  mm(c, n, D2 * x, x, t.Q, x, false, b.bTr, (int64_t)D2 * x, false, b.bV3, (int64_t)D2 * x);
  // V3[alpha][(k,l)][nu] = sum_m a[k][l][m] V2[(alpha,m)][nu]
  gemm(s, f, D2, x, (int)g.D4, Operand{a, D2, true, 0}, Operand{b.bV3, x, false, g.D4 * x},
       Output{b.bV2, x, f, (int64_t)D2 * x}, x, 1, 1.0, 0.0, c->ws);
  gemm(s, f, (int)g.D4, D2, x, Operand{b.bV3, x, false, g.D4 * x},
       Operand{t.V2, x, true, (int64_t)D2 * x}, Output{b.abpart, D2, f, g.D6}, x, 1, 1.0, 0.0,
       c->ws);
  launch_sum_batches(s, b.abpart, x, g.D6, b.ab, 1.0);
  // V2 = V Q
  mm(c, n, x, n, t.V, n, true, b.bV2, x, false, b.bQ, x, 1.0, 1.0);
  mm(c, n, n, x, b.bV2, x, false, t.Q, x, true, b.bV, n);
  // Cq = Q^T Ct Q (bCq symmetric)
  mm(c, n, x, x, t.Gm, x, false, b.bCq, x, false, b.bQ, x, 2.0, 1.0);
  mm(c, n, x, x, t.Q, x, false, b.bCq, x, false, b.QC, x);
  mm(c, n, n, x, b.QC, x, false, t.Q, x, true, b.bCt, n);
  proj_bwd(c, P, oP);
  ct_bwd_w(c, true);
  ct_bwd_v(c, C, T, oC, oT);
}

// Bond energy of the tape's state (Sec. II.C, Fig. 4b: the six-corner ring
// with the apex pair open) and its adjoint: writes e to eout[0], the state
// cotangents to (oC, oT, oP), the double-layer cotangents to ab (+=), aOb
// and aOrb.
void energy_vjp(ctm_ctx* c, const double* C, const double* T, const double* P, double* oC,
                double* oT, double* oP) {
  const Dims g = dims_of(c);
  const int x = g.x, D2 = g.D2, n = g.n, dd = g.dd;
  GradBuffers& b = *c->grad;
  const Tape& t = b.tp;
  hipStream_t s = c->stream;
  const DType f = DType::F64;
  const int x2 = x * x;
  const int64_t D2dd = (int64_t)D2 * dd;
  // forward: Env = Q Cr^5 Q^T with Cr = Q^T Ct Q / max|.|
  launch_maxabs_scale(s, t.Cq, b.Cr, t.sc + 3, x);
  mm(c, x, x, x, b.Cr, x, false, b.Cr, x, false, b.Cr2, x);
  mm(c, x, x, x, b.Cr2, x, false, b.Cr2, x, false, b.Cr4, x);
  mm(c, x, x, x, b.Cr4, x, false, b.Cr, x, false, b.Cr5, x);
  mm(c, n, x, x, t.Q, x, false, b.Cr5, x, false, b.QC5, x);
  gemm(s, f, D2, D2, x, Operand{t.Q, x, false, (int64_t)D2 * x, 0},
       Operand{b.QC5, x, true, 0, (int64_t)D2 * x}, Output{b.EnvP, D2, f, (int64_t)x * g.D4, g.D4},
       x, x, 1.0, 0.0, c->ws);
  gemm(s, f, D2, D2, x, Operand{T, x, false, (int64_t)D2 * x, 0},
       Operand{t.TCp, D2, false, 0, (int64_t)x * D2},
       Output{b.TCTp, D2, f, (int64_t)x * g.D4, g.D4}, x, x, 1.0, 0.0, c->ws);
  mm(c, x2, (int)D2dd, (int)g.D4, b.TCTp, g.D4, false, c->aO, D2dd, false, b.XO, D2dd);
  mm(c, x2, (int)D2dd, (int)g.D4, b.EnvP, g.D4, false, c->aOr, D2dd, false, b.EO, D2dd);
  mm(c, dd, dd, x2 * D2, b.XO, dd, true, b.EO, dd, false, b.R, dd);
  launch_energy_bwd(s, b.R, b.h, g.d, b.eout, b.Rb);
  // R = XO^T EO
  mm(c, x2 * D2, dd, dd, b.EO, dd, false, b.Rb, dd, true, b.bXO, dd);
  mm(c, x2 * D2, dd, dd, b.XO, dd, false, b.Rb, dd, false, b.bEO, dd);
  // XO = TCTp aO: bTCTp (held in bV), aOb
  double* bTCTp = b.bV;
  mm(c, x2, (int)g.D4, (int)D2dd, b.bXO, D2dd, false, c->aO, D2dd, true, bTCTp, g.D4);
  mm(c, (int)g.D4, (int)D2dd, x2, b.TCTp, g.D4, true, b.bXO, D2dd, false, b.aOb, D2dd);
  // TCTp[a][b][I][J] = (T C T^T)[(a,I)][(b,J)] = sum_g T[(a,I)][g] TCpT[g][(b,J)]
  double* bTCT = b.bCt;
  launch_swap_mid(s, bTCTp, bTCT, x, x, D2, D2, false);  // -> [(a,I)][(b,J)]
  launch_swap_mid(s, t.TCp, b.TCpT, 1, x, x, D2, false);  // TCp[b][g][J] -> TCpT[g][b][J]
  mm(c, n, x, n, bTCT, n, false, b.TCpT, n, true, b.bTe, x);
  mm(c, x, n, n, T, x, true, bTCT, n, false, b.bTCpT, n);
  // EO = EnvP aOr: bEnvP (held in bV3), aOrb
  double* bEnvP = b.bV3;
  mm(c, x2, (int)g.D4, (int)D2dd, b.bEO, D2dd, false, c->aOr, D2dd, true, bEnvP, g.D4);
  mm(c, (int)g.D4, (int)D2dd, x2, b.EnvP, g.D4, true, b.bEO, D2dd, false, b.aOrb, D2dd);
  // EnvP[a][b][K][L] = sum_nu Q[(a,K)][nu] QC5[(b,L)][nu]
  double* E2 = b.bCtP;
  launch_swap_mid(s, bEnvP, E2, x, x, D2, D2, false);  // -> [(a,K)][(b,L)]
  mm(c, n, x, n, E2, n, false, b.QC5, x, false, b.bQ, x);
  mm(c, n, x, n, E2, n, true, t.Q, x, false, b.bQC5, x);
  // QC5 = Q Cr^5
  mm(c, n, x, x, b.bQC5, x, false, b.Cr5, x, true, b.bQ, x, 1.0, 1.0);
  mm(c, x, x, n, t.Q, x, true, b.bQC5, x, false, b.bCr5, x);
  // Cr5 = Cr4 Cr, Cr4 = Cr2 Cr2, Cr2 = Cr Cr
  mm(c, x, x, x, b.bCr5, x, false, b.Cr, x, true, b.bCr4, x);
  mm(c, x, x, x, b.Cr4, x, true, b.bCr5, x, false, b.bCr, x);
  mm(c, x, x, x, b.bCr4, x, false, b.Cr2, x, true, b.bCr2, x);
  mm(c, x, x, x, b.Cr2, x, true, b.bCr4, x, false, b.bCr2, x, 1.0, 1.0);
  mm(c, x, x, x, b.bCr2, x, false, b.Cr, x, true, b.bCr, x, 1.0, 1.0);
  mm(c, x, x, x, b.Cr, x, true, b.bCr2, x, false, b.bCr, x, 1.0, 1.0);
  // Cr = Cq / max|Cq| (the scale cancels in rho), Cq = Q^T Ct Q
  launch_div_scalar(s, b.bCr, t.sc + 3, b.bCq, (int64_t)x * x);
  launch_sym_scaled(s, b.bCq, nullptr, 1.0, b.Mx, x);
  mm(c, n, x, x, t.Gm, x, false, b.Mx, x, false, b.bQ, x, 1.0, 1.0);
  mm(c, n, x, x, t.Q, x, false, b.bCq, x, false, b.QC, x);
  mm(c, n, n, x, b.QC, x, false, t.Q, x, true, b.bCt, n);
  proj_bwd(c, P, oP);
  ct_bwd_w(c, false);
  launch_swap_mid(s, b.bTCpT, b.bTCp, 1, x, x, D2, true);  // += [g][b][J] -> [b][g][J]
  ct_bwd_v(c, C, T, oC, oT);
  launch_axpy(s, b.bTe, oT, g.NT, 1.0);
}

// Squared norms of the last increment of the double-layer cotangent and of
// the cotangent itself (host values; synchronizes).  abprev is overwritten.
void increment_norms(ctm_ctx* c, double* inc2, double* tot2) {
  const Dims g = dims_of(c);
  GradBuffers& b = *c->grad;
  hipStream_t s = c->stream;
  launch_axpy(s, b.ab, b.abprev, g.D6, -1.0);  // abprev <- abprev - ab
  launch_dot(s, b.abprev, b.abprev, g.D6, b.parts, b.dots + 1);
  launch_dot(s, b.ab, b.ab, g.D6, b.parts, b.dots + 2);
  double h[2];
  CTM_HIP(hipMemcpyAsync(h, b.dots + 1, sizeof(h), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipStreamSynchronize(s));
  *inc2 = h[0];
  *tot2 = h[1];
}

}  // namespace

// Largest change of the (unit-norm) corner under one step that mode 0
// accepts as stationary.
constexpr double kStationaryCorner = 1e-5;

int do_grad(ctm_ctx* c, const double* h_host, int mode, double tol, int max_iter, double* gradA_dev,
            double* e_host, int* iters_host) {
  if (!h_host || !gradA_dev || mode < 0 || max_iter < 0)
    throw std::invalid_argument("ctm_grad: bad arguments");
  const Dims g = dims_of(c);
  if (c->chi_c != c->chi || c->p_rows != g.n || g.n <= g.x) {
    c->err = "ctm_grad needs a truncated environment (chi_c = chi, chi D^2 > chi and a projector)";
    return CTM_ESTATE;
  }
  ensure_energy_buffers(c);
  ensure_grad_buffers(c);
  GradBuffers& b = *c->grad;
  hipStream_t s = c->stream;
  const int x = g.x, n = g.n;
  const int64_t x2 = (int64_t)x * x, nx = (int64_t)n * x;
  CTM_HIP(hipMemcpyAsync(b.h, h_host, (size_t)g.dd * g.dd * sizeof(double), hipMemcpyHostToDevice,
                         s));
  launch_zero(s, b.ab, g.D6);
  int iters = 0;
  bool converged = true;
  if (mode == 0) {
    tape_forward(c, c->C, c->T, c->P);
    // The series assumes a fixed point element by element.  Where the corner
    // spectrum has +-lambda pairs, C keeps turning within their
    // two-dimensional eigenspaces while T, P, the spectrum and the energy
    // converge; one step then changes C by O(max |C|) and the series does
    // not converge.  Refuse such a state (the unrolled mode handles it).
    {
      std::vector<double> c0((size_t)x2), c1((size_t)x2);
      CTM_HIP(hipMemcpyAsync(c0.data(), c->C, (size_t)x2 * sizeof(double), hipMemcpyDeviceToHost, s));
      CTM_HIP(hipMemcpyAsync(c1.data(), b.tp.Cn, (size_t)x2 * sizeof(double), hipMemcpyDeviceToHost,
                             s));
      CTM_HIP(hipStreamSynchronize(s));
      double dc = 0.0;
      for (int64_t i = 0; i < x2; ++i) dc = std::max(dc, std::fabs(c1[i] - c0[i]));
      if (!(dc <= kStationaryCorner)) {
        c->err = "ctm_grad mode 0 needs a stationary environment, but one step changes the corner by " +
                 std::to_string(dc) +
                 " (the corner keeps turning within +-lambda pairs of its spectrum); use mode k > 0";
        return CTM_ESTATE;
      }
    }
    energy_vjp(c, c->C, c->T, c->P, b.xC[0], b.xT[0], b.xP[0]);
    int cur = 0;
    converged = false;
    while (iters < max_iter) {
      launch_copy(s, b.ab, b.abprev, g.D6);
      step_vjp(c, c->C, c->T, c->P, b.xC[cur], b.xT[cur], b.xP[cur], b.xC[cur ^ 1], b.xT[cur ^ 1],
               b.xP[cur ^ 1]);
      cur ^= 1;
      ++iters;
      double inc2, tot2;
      increment_norms(c, &inc2, &tot2);
      if (!std::isfinite(inc2) || !std::isfinite(tot2)) {
        c->err = "adjoint iteration produced non-finite values";
        return CTM_ENONFINITE;
      }
      if (inc2 <= tol * tol * tot2) {
        converged = true;
        break;
      }
    }
  } else {
    const int k = mode;
    while ((int)b.ckC.size() < k + 1) {
      b.ckC.push_back(c->allocd(x2));
      b.ckT.push_back(c->allocd(g.NT));
      b.ckP.push_back(c->allocd(nx));
    }
    launch_copy(s, c->C, b.ckC[0], x2);
    launch_copy(s, c->T, b.ckT[0], g.NT);
    launch_copy(s, c->P, b.ckP[0], nx);
    for (int i = 0; i < k; ++i) {
      tape_forward(c, b.ckC[i], b.ckT[i], b.ckP[i]);
      launch_copy(s, b.tp.Cn, b.ckC[i + 1], x2);
      launch_copy(s, b.tp.Tn, b.ckT[i + 1], g.NT);
      launch_copy(s, b.tp.Q, b.ckP[i + 1], nx);
    }
    tape_forward(c, b.ckC[k], b.ckT[k], b.ckP[k]);
    energy_vjp(c, b.ckC[k], b.ckT[k], b.ckP[k], b.xC[0], b.xT[0], b.xP[0]);
    int cur = 0;
    for (int i = k - 1; i >= 0; --i) {
      tape_forward(c, b.ckC[i], b.ckT[i], b.ckP[i]);
      step_vjp(c, b.ckC[i], b.ckT[i], b.ckP[i], b.xC[cur], b.xT[cur], b.xP[cur], b.xC[cur ^ 1],
               b.xT[cur ^ 1], b.xP[cur ^ 1]);
      cur ^= 1;
      ++iters;
    }
  }
  // dE/dA through the double layers, projected onto the symmetric subspace
  launch_zero(s, b.gA, (int64_t)g.d * c->D * c->D * c->D);
  launch_double_layer_bwd(s, b.ab, c->A, g.d, c->D, b.gA);
  launch_double_layer_open_bwd(s, b.aOb, c->A, g.d, c->D, 0, b.gA);
  launch_double_layer_open_bwd(s, b.aOrb, c->A, g.d, c->D, 1, b.gA);
  launch_symmetrize_plain(s, b.gA, gradA_dev, g.d, c->D);
  double e = 0.0;
  CTM_HIP(hipMemcpyAsync(&e, b.eout, sizeof(double), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipStreamSynchronize(s));
  if (e_host) *e_host = e;
  if (iters_host) *iters_host = iters;
  if (!converged) {
    c->err = "adjoint series did not reach tol in max_iter iterations";
    return CTM_ENOTCONV;
  }
  return CTM_OK;
}

}  // namespace ctm
