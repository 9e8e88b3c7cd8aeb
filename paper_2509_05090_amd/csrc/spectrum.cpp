// Corner spectrum for the convergence test (host, FP64).
//
// The corner is small (chi x chi) and the test runs every few steps, on a
// copy taken after the stream is synchronized.  Eigenvalues of the real
// symmetric matrix: Householder reduction to tridiagonal form (Golub & Van
// Loan, Matrix Computations, Sec. 8.3.1; the symmetric updates on the lower
// triangle only), then the symmetric QR iteration with implicit Wilkinson
// shifts (Alg. 8.3.2, 8.3.3), O(n^2) for all eigenvalues.  Bisection on
// Sturm sequence counts (Sec. 8.4.1) remains as the fallback should the
// iteration not settle.
#include "spectrum.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <numeric>

namespace ctm {

namespace {

// Reduce the symmetric n x n matrix A (row-major, overwritten; only the
// lower triangle is read and updated) to tridiagonal form: diagonal d[0..n),
// off-diagonal e[0..n-1).
void tridiagonalize(std::vector<double>& A, int n, std::vector<double>& d,
                    std::vector<double>& e) {
  auto at = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  std::vector<double> v(n), p(n), w(n);
  d.assign(n, 0.0);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    const int o = k + 1;      // first row / column of the trailing block B
    double xn = 0.0;
    for (int i = 0; i < m; ++i) xn += at(o + i, k) * at(o + i, k);
    xn = std::sqrt(xn);
    const double x0 = at(o, k);
    if (xn == 0.0) continue;
    const double alpha = x0 > 0.0 ? -xn : xn;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = at(o + i, k) - (i == 0 ? alpha : 0.0);
      vv += v[i] * v[i];
    }
    if (vv == 0.0) continue;
    // p = (2/vv) B v from the lower triangle of B; w = p - (v^T p / vv) v.
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double* row = &at(o + i, o);
      double t = row[i] * v[i];
      const double vi = v[i];
      for (int j = 0; j < i; ++j) {
        t += row[j] * v[j];
        p[j] += row[j] * vi;
      }
      p[i] += t;
    }
    for (int i = 0; i < m; ++i) p[i] *= 2.0 / vv;
    double vp = 0.0;
    for (int i = 0; i < m; ++i) vp += v[i] * p[i];
    const double K = vp / vv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    // B -= v w^T + w v^T on the lower triangle
    for (int i = 0; i < m; ++i) {
      double* row = &at(o + i, o);
      const double vi = v[i], wi = w[i];
      for (int j = 0; j <= i; ++j) row[j] -= vi * w[j] + wi * v[j];
    }
    at(o, k) = alpha;
  }
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
}

// One implicit symmetric QR step with Wilkinson shift on the unreduced
// block [p, q] of the tridiagonal (d, e) (Golub & Van Loan, Alg. 8.3.2).
// The rotation in plane (k, k+1) is G = [c -s; s c] with G^T (x, z) = (r, 0):
// at k = p, (x, z) is the shifted first column; afterwards x = T(k, k-1) and
// z the bulge T(k+1, k-1) left by the previous rotation.
void implicit_qr_step(std::vector<double>& d, std::vector<double>& e, int p, int q) {
  const double t2 = e[q - 1] * e[q - 1];
  const double h = 0.5 * (d[q - 1] - d[q]);
  const double den = h + std::copysign(std::sqrt(h * h + t2), h == 0.0 ? 1.0 : h);
  const double mu = den == 0.0 ? d[q] : d[q] - t2 / den;
  double x = d[p] - mu, z = e[p];
  for (int k = p; k < q; ++k) {
    const double r = std::hypot(x, z);
    const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
    if (k > p) e[k - 1] = r;
    const double a = d[k], b = e[k], dd = d[k + 1];
    d[k] = c * c * a + 2.0 * c * s * b + s * s * dd;
    d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * dd;
    e[k] = c * s * (dd - a) + (c * c - s * s) * b;
    if (k + 1 < q) {
      x = e[k];
      z = s * e[k + 1];  // new bulge T(k+2, k)
      e[k + 1] *= c;
    }
  }
}

// Eigenvalues of the tridiagonal (d, e) by the symmetric QR iteration
// (Golub & Van Loan, Alg. 8.3.3): off-diagonals below eps (|d_i| + |d_i+1|)
// are set to zero and the trailing unreduced block takes an implicit step
// until the matrix is diagonal.  False if it has not settled after 30 n
// steps.
bool tridiag_qr_eigenvalues(std::vector<double> d, std::vector<double> e,
                            std::vector<double>& out) {
  const int n = (int)d.size();
  int q = n - 1, steps = 0;
  while (q > 0) {
    for (int i = 0; i < q; ++i)
      if (std::fabs(e[i]) <= DBL_EPSILON * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    while (q > 0 && e[q - 1] == 0.0) --q;
    if (q == 0) break;
    int p = q - 1;
    while (p > 0 && e[p - 1] != 0.0) --p;
    if (++steps > 30 * n) return false;
    implicit_qr_step(d, e, p, q);
  }
  std::sort(d.begin(), d.end());
  out = std::move(d);
  return true;
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
  std::vector<double> ev;
  if (tridiag_qr_eigenvalues(d, e, ev)) return ev;
  double lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  ev.assign(n, 0.0);
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

namespace {

// Gershgorin interval of the tridiagonal matrix.
void gershgorin(const std::vector<double>& d, const std::vector<double>& e, double& lo, double& hi) {
  const int n = (int)d.size();
  lo = hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
}

// Solve (T - lam I) y = b in place by Gaussian elimination with partial
// pivoting on the tridiagonal (rows swap with their successor only); zero
// pivots are replaced by a tiny multiple of the matrix scale.
void tridiag_shifted_solve(const std::vector<double>& d, const std::vector<double>& e, double lam,
                           double tiny, std::vector<double>& b) {
  const int n = (int)d.size();
  // row i of the current (possibly swapped) system: a[i] (diag), u1[i], u2[i] (fill-in)
  std::vector<double> a(n), u1(n, 0.0), u2(n, 0.0), sub(n, 0.0);
  for (int i = 0; i < n; ++i) a[i] = d[i] - lam;
  for (int i = 0; i + 1 < n; ++i) {
    u1[i] = e[i];
    sub[i + 1] = e[i];
  }
  for (int i = 0; i + 1 < n; ++i) {
    // eliminate sub[i+1] (entry (i+1, i)) using row i or swapped row i+1
    if (std::fabs(sub[i + 1]) > std::fabs(a[i])) {
      // swap rows i and i+1 (row i+1 has entries at i, i+1, i+2)
      const double r0 = sub[i + 1], r1 = a[i + 1], r2 = i + 2 < n ? u1[i + 1] : 0.0;
      const double s0 = a[i], s1 = u1[i], s2 = u2[i];
      a[i] = r0;
      u1[i] = r1;
      u2[i] = r2;
      std::swap(b[i], b[i + 1]);
      const double m = s0 / r0;
      a[i + 1] = s1 - m * r1;
      if (i + 2 < n) u1[i + 1] = s2 - m * r2;
      b[i + 1] -= m * b[i];
    } else {
      if (a[i] == 0.0) a[i] = tiny;
      const double m = sub[i + 1] / a[i];
      a[i + 1] -= m * u1[i];
      if (i + 2 < n) u1[i + 1] -= m * u2[i];
      b[i + 1] -= m * b[i];
    }
  }
  if (a[n - 1] == 0.0) a[n - 1] = tiny;
  for (int i = n - 1; i >= 0; --i) {
    double t = b[i];
    if (i + 1 < n) t -= u1[i] * b[i + 1];
    if (i + 2 < n) t -= u2[i] * b[i + 2];
    b[i] = t / (a[i] == 0.0 ? tiny : a[i]);
  }
}

}  // namespace

double tridiag_eigenvalue(const std::vector<double>& d, const std::vector<double>& e, int j) {
  double lo, hi;
  gershgorin(d, e, lo, hi);
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  double a = lo, b = hi;
  for (int it = 0; it < 300; ++it) {
    const double mid = 0.5 * (a + b);
    if (b - a <= 2.0 * DBL_EPSILON * scale || mid == a || mid == b) break;
    if (count_below(d, e, mid) > j)
      b = mid;
    else
      a = mid;
  }
  return 0.5 * (a + b);
}

void tridiag_top_eigenpairs(const std::vector<double>& d, const std::vector<double>& e, int k,
                            std::vector<double>& lam, std::vector<double>& z) {
  const int n = (int)d.size();
  // candidates: the k smallest and the k largest eigenvalues (by ascending index)
  std::vector<int> idx;
  for (int j = 0; j < std::min(k, n); ++j) idx.push_back(j);
  for (int j = std::max(k, n - k); j < n; ++j) idx.push_back(j);
  std::vector<double> val(idx.size());
  for (size_t t = 0; t < idx.size(); ++t) val[t] = tridiag_eigenvalue(d, e, idx[t]);
  std::vector<int> ord(idx.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int p, int q) {
    if (std::fabs(val[p]) != std::fabs(val[q])) return std::fabs(val[p]) > std::fabs(val[q]);
    if (val[p] != val[q]) return val[p] > val[q];
    return idx[p] < idx[q];
  });
  lam.resize(k);
  for (int t = 0; t < k; ++t) lam[t] = val[ord[t]];
  double lo, hi;
  gershgorin(d, e, lo, hi);
  const double tnorm = std::max(std::fabs(lo), std::fabs(hi));
  const double tiny = DBL_EPSILON * std::max(tnorm, DBL_MIN);
  const double cluster = 1e-3 * tnorm;
  z.assign((size_t)n * k, 0.0);
  std::vector<std::vector<double>> vecs;
  uint64_t state = 0x9E3779B97F4A7C15ull;
  for (int t = 0; t < k; ++t) {
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {  // deterministic start vector (splitmix64 draws in (-1, 1))
      state += 0x9E3779B97F4A7C15ull;
      uint64_t v = state;
      v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
      v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
      v ^= v >> 31;
      y[i] = (double)(v >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    for (int it = 0; it < 4; ++it) {
      tridiag_shifted_solve(d, e, lam[t], tiny, y);
      for (int q = 0; q < t; ++q)
        if (std::fabs(lam[q] - lam[t]) < cluster) {
          double dot = 0.0;
          for (int i = 0; i < n; ++i) dot += vecs[q][i] * y[i];
          for (int i = 0; i < n; ++i) y[i] -= dot * vecs[q][i];
        }
      double nr = 0.0;
      for (double v : y) nr += v * v;
      nr = std::sqrt(nr);
      for (double& v : y) v /= nr;
    }
    vecs.push_back(y);
    for (int i = 0; i < n; ++i) z[(size_t)i * k + t] = y[i];
  }
}

}  // namespace ctm
