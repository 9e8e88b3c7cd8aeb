// Thin QR factorization of a tall FP64 matrix by blocked Householder
// reflections, for the projector of the QR-based CTMRG.
//
// The matrix is processed in panels of NB columns (NB = 32, or 16 for more
// than 8192 rows).  A panel is factored as a tall-skinny QR (TSQR): its rows
// are split into L row blocks ("leaves"), each leaf is factored by one
// workgroup with the block held in registers, and the L stacked triangular
// factors are factored once more by the last leaf workgroup to finish (the
// "tree").  The panel's orthogonal factor is therefore Q_p = Q_L Q_T: Q_L
// block diagonal over the leaves, Q_T acting on the stacked top rows of the
// leaves, each a product of Householder reflections in compact WY form
// I - Y T Y^T.  Trailing columns are updated with Q_p^T, and the explicit Q
// is accumulated backwards.
#pragma once
#include "gemm.hpp"

namespace ctm {

constexpr int QR_NB_MAX = 32;
constexpr int QR_MAX_LEAVES = 32;
constexpr int QR_MAX_STACK = QR_MAX_LEAVES * QR_NB_MAX;
constexpr int QR_MAX_ROWS = 32768;  // largest n accepted

// Row blocking of one panel (host side).
struct QrPanel {
  int nb;          // panel width of this factorization (32 or 16)
  int j0, w;       // first column, width (w <= nb)
  int L, rpl;      // leaves, rows per leaf (the last one may have fewer)
  int tr_leaf;     // register rows per lane group in the leaf workgroups (16 tr rows each)
  int tr_tree;     // register rows per lane group in the stacked factorization
};

// Device workspace of one factorization.  Carved from one allocation of
// qr_work_bytes(n, k) bytes by qr_work_carve(); `counter` must be zero
// before the first use (the kernels leave it zero).
struct QrWork {
  int n = 0, k = 0;
  double* Y = nullptr;    // n x k: leaf Householder vectors of panel p at rows [j0, n), cols [j0, j0+w)
  double* Tl = nullptr;   // per panel: QR_MAX_LEAVES leaf WY factors (nb x nb)
  double* Yt = nullptr;   // per panel: stacked-row Householder vectors (QR_MAX_LEAVES nb x nb)
  double* Tt = nullptr;   // per panel: stacked WY factor (nb x nb)
  double* S = nullptr;    // stacked leaf R factors (QR_MAX_STACK x nb)
  unsigned* counter = nullptr;  // per panel: leaves finished (reset by the tree workgroup)
};

size_t qr_work_bytes(int n, int k);
// Carves the workspace and clears the counters (enqueued on s).
QrWork qr_work_carve(hipStream_t s, void* p, int n, int k);

// Panel plan of an n x k factorization (n >= k, n <= QR_MAX_ROWS).
QrPanel qr_panel_plan(int n, int k, int j0);

// Factor M (n x k, row-major with leading dimension ld, n >= k) in place:
// R in the upper triangle of the first k rows (zeros below it within the
// first k rows); the reflectors go to w.  R's diagonal signs follow the
// stacked factorization, not LAPACK's convention.
// With kx > k, columns [k, kx) of M are carried along: every panel's
// trailing update applies to them too, so that they end up as Q^T B for
// their input B (Q the full n x n orthogonal factor); their first k rows
// are then Q1^T B, Q1 = the thin factor of householder_form_q().
void householder_qr(hipStream_t s, double* M, int ld, int n, int k, QrWork& w, int kx = -1);

// Explicit Q (n x k, leading dimension ldq) of the last householder_qr().
void householder_form_q(hipStream_t s, const QrWork& w, int n, int k, double* Q, int ldq);

}  // namespace ctm
