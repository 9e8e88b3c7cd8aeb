// Corner spectrum for the convergence test (host, FP64).
//
// The corner is small (chi x chi) and the test runs every few steps, on a
// copy taken after the stream is synchronized.  Eigenvalues of the real
// symmetric matrix: Householder reduction to tridiagonal form, then
// bisection on Sturm sequence counts (Golub & Van Loan, Matrix
// Computations, Secs. 8.3.1 and 8.4.1).
#include "spectrum.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace ctm {

namespace {

// Reduce the symmetric n x n matrix A (row-major, overwritten) to
// tridiagonal form: diagonal d[0..n), off-diagonal e[0..n-1).
void tridiagonalize(std::vector<double>& A, int n, std::vector<double>& d,
                    std::vector<double>& e) {
  auto at = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  std::vector<double> v(n), p(n), w(n);
  d.assign(n, 0.0);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double xn = 0.0;
    for (int i = 0; i < m; ++i) xn += at(k + 1 + i, k) * at(k + 1 + i, k);
    xn = std::sqrt(xn);
    const double x0 = at(k + 1, k);
    if (xn == 0.0) continue;
    const double alpha = x0 > 0.0 ? -xn : xn;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = at(k + 1 + i, k) - (i == 0 ? alpha : 0.0);
      vv += v[i] * v[i];
    }
    if (vv == 0.0) continue;
    // p = (2/vv) B v with B the trailing block; w = p - (v^T p / vv) v.
    for (int i = 0; i < m; ++i) {
      double t = 0.0;
      for (int j = 0; j < m; ++j) t += at(k + 1 + i, k + 1 + j) * v[j];
      p[i] = 2.0 * t / vv;
    }
    double vp = 0.0;
    for (int i = 0; i < m; ++i) vp += v[i] * p[i];
    const double K = vp / vv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) at(k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
    at(k + 1, k) = alpha;
    at(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) at(k + 1 + i, k) = at(k, k + 1 + i) = 0.0;
  }
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
}

// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm count via
// the pivots of the LDL^T factorization of T - x I).
int count_below(const std::vector<double>& d, const std::vector<double>& e, double x) {
  const int n = (int)d.size();
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    if (q == 0.0) q = -DBL_MIN;
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

}  // namespace

std::vector<double> symmetric_eigenvalues(std::vector<double> A, int n) {
  if (n <= 0) return {};
  if (n == 1) return {A[0]};
  std::vector<double> d, e;
  tridiagonalize(A, n, d, e);
  double lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  std::vector<double> ev(n);
  for (int j = 0; j < n; ++j) {
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (b - a <= 2.0 * DBL_EPSILON * scale || mid == a || mid == b) break;
      if (count_below(d, e, mid) > j)
        b = mid;
      else
        a = mid;
    }
    ev[j] = 0.5 * (a + b);
  }
  return ev;
}

std::vector<double> normalized_spectrum(const std::vector<double>& C, int n) {
  std::vector<double> ev = symmetric_eigenvalues(C, n);
  for (double& x : ev) x = std::fabs(x);
  std::sort(ev.begin(), ev.end(), [](double a, double b) { return a > b; });
  const double m = ev.empty() ? 0.0 : ev[0];
  if (m > 0.0)
    for (double& x : ev) x /= m;
  return ev;
}

double spectrum_change(const std::vector<double>& s, const std::vector<double>& prev) {
  const size_t m = std::max(s.size(), prev.size());
  double c = 0.0;
  for (size_t i = 0; i < m; ++i) {
    const double a = i < s.size() ? s[i] : 0.0, b = i < prev.size() ? prev[i] : 0.0;
    c = std::max(c, std::fabs(a - b));
  }
  return c;
}

}  // namespace ctm
