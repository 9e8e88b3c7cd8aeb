// Eigenvectors of the symmetric enlarged corner for the conventional
// eigendecomposition projector (Sec. II.B, Fig. 3c): FP64 Householder
// tridiagonalization on the GPU with the orthogonal factor accumulated, the
// tridiagonal eigenproblem for the wanted eigenpairs on the host, and the
// back-transformation as one matrix product.
#pragma once
#include <vector>

#include "gemm.hpp"

namespace ctm {

struct EvdWork {
  int n = 0, k = 0;
  double* A = nullptr;    // n x n working copy (destroyed)
  double* Q = nullptr;    // n x n accumulated orthogonal factor
  double* v = nullptr;    // n: current reflector
  double* p = nullptr;    // n: tau A v
  double* q = nullptr;    // n: Q v
  double* d = nullptr;    // n: diagonal of the tridiagonal matrix
  double* e = nullptr;    // n: off-diagonal
  double* scal = nullptr; // 8 scalars
  double* Z = nullptr;    // n x k tridiagonal eigenvectors
  double* sgn = nullptr;  // k column signs
};

size_t evd_work_bytes(int n, int k);
EvdWork evd_work_carve(void* p, int n, int k);

// A_in (n x n symmetric, row-major, element type t) = Q tri(d, e) Q^T:
// the copy in w.A is reduced, w.Q accumulates Q = H_0 H_1 ... H_{n-3}, and d,
// e are left in device memory.
void tridiagonalize(hipStream_t s, const void* A_in, DType t, int n, EvdWork& w);

// Eigenvectors of the k eigenvalues of largest magnitude of the symmetric
// n x n A_in (order: decreasing |lambda|, then larger lambda, then lower
// ascending index) into U (n x k, leading dimension ldu); eigenvalues to
// lam_host.  Column signs: if P (n x k, ld k) is non-null, each column has a
// non-negative overlap with P's column; otherwise each column's entry of
// largest magnitude (lowest row on ties) is positive.  Synchronizes s.
void eigh_top(hipStream_t s, const void* A_in, DType t, int n, int k, EvdWork& w, const Scratch& ws,
              double* U, int ldu, const double* P, std::vector<double>& lam_host);

}  // namespace ctm
