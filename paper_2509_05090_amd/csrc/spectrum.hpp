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

}  // namespace ctm
