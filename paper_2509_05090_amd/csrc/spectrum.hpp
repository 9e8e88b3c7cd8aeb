// Corner spectrum for the convergence test (host, FP64).
#pragma once
#include <vector>

namespace ctm {

// Eigenvalues (ascending) of the real symmetric n x n row-major matrix A.
std::vector<double> symmetric_eigenvalues(std::vector<double> A, int n);

// |eigenvalues| of the symmetric corner in decreasing order, divided by the largest.
std::vector<double> normalized_spectrum(const std::vector<double>& C, int n);

// Max-norm distance of two spectra, the shorter padded with zeros.
double spectrum_change(const std::vector<double>& s, const std::vector<double>& prev);

// Symmetric tridiagonal matrix: diagonal d (n), off-diagonal e (n - 1).
// Eigenvalue number j (ascending, 0-based) by bisection on Sturm counts.
double tridiag_eigenvalue(const std::vector<double>& d, const std::vector<double>& e, int j);

// Eigenpairs of the k eigenvalues of largest magnitude, ordered by
// decreasing |lambda|, then larger lambda, then lower ascending index:
// lam (k) and the eigenvectors z (n x k, row-major, unit norm), by inverse
// iteration with reorthogonalization inside clusters of close eigenvalues.
void tridiag_top_eigenpairs(const std::vector<double>& d, const std::vector<double>& e, int k,
                            std::vector<double>& lam, std::vector<double>& z);

}  // namespace ctm
