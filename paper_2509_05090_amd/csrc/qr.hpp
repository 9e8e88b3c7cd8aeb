// Thin QR factorization of a tall FP64 matrix by blocked Householder
// reflections (compact WY form), for the projector of the QR-based CTMRG.
#pragma once
#include "gemm.hpp"

namespace ctm {

constexpr int QR_NB = 16;  // panel width

struct QrWork {
  double* Y = nullptr;    // n x k explicit Householder vectors (unit diagonal, zeros above)
  double* tau = nullptr;  // k
  double* Tf = nullptr;   // ceil(k/NB) blocks of NB x NB upper-triangular WY factors
  double* W = nullptr;    // NB x k product buffer
  double* W2 = nullptr;   // NB x k product buffer
  Scratch ws;             // split-K scratch for NB x k products
};

// Factor M (n x k, row-major with leading dimension ld, n >= k) in place:
// R in the upper triangle, Householder vectors below it (and in w.Y).
void householder_qr(hipStream_t s, double* M, int ld, int n, int k, QrWork& w);

// Explicit Q (n x k, leading dimension ldq) of the last householder_qr().
void householder_form_q(hipStream_t s, const QrWork& w, int n, int k, double* Q, int ldq);

}  // namespace ctm
