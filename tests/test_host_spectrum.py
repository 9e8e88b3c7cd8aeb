"""The library's host eigenvalue routine for the convergence test (Householder
tridiagonalization, then the symmetric QR iteration with implicit Wilkinson
shifts; bisection as fallback), built from its source with the host
compiler and compared with LAPACK's symmetric eigenvalues (numpy.linalg.eigvalsh)
on random, +-lambda-paired (as the converged corners have), threefold
degenerate, diagonal, tridiagonal, zero and widely scaled spectra."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_05090_amd", "csrc")
WRAP = r'''
#include "spectrum.hpp"
#include <cstring>
extern "C" void eig(const double* A, int n, double* out) {
  std::vector<double> a(A, A + (size_t)n * n);
  auto ev = ctm::symmetric_eigenvalues(a, n);
  std::memcpy(out, ev.data(), (size_t)n * sizeof(double));
}
extern "C" void spec(const double* C, int n, double* out) {
  std::vector<double> c(C, C + (size_t)n * n);
  auto s = ctm::normalized_spectrum(c, n);
  std::memcpy(out, s.data(), (size_t)n * sizeof(double));
}
'''


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("spec")
    (d / "wrap.cpp").write_text(WRAP)
    so = d / "libspec.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, "-o", str(so),
                    str(d / "wrap.cpp"), os.path.join(CSRC, "spectrum.cpp")], check=True)
    return ctypes.CDLL(str(so))


def _call(lib, fn, A):
    n = A.shape[0]
    out = np.zeros(n)
    A = np.ascontiguousarray(A, dtype=np.float64)
    getattr(lib, fn)(A.ctypes.data_as(ctypes.c_void_p), n, out.ctypes.data_as(ctypes.c_void_p))
    return out


def _case(rng, n, kind):
    def rotate(w):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = (Q * w) @ Q.T
        return (A + A.T) / 2
    if kind == "random":
        X = rng.standard_normal((n, n))
        return X + X.T
    if kind == "pm_pairs":
        lam = np.abs(rng.standard_normal(n // 2 + 1))
        return rotate(np.concatenate([lam, -lam])[:n])
    if kind == "degenerate":
        return rotate(np.repeat(rng.standard_normal((n + 2) // 3), 3)[:n])
    if kind == "diagonal":
        return np.diag(rng.standard_normal(n))
    if kind == "tridiagonal":
        off = rng.standard_normal(max(n - 1, 0))
        return np.diag(rng.standard_normal(n)) + np.diag(off, 1) + np.diag(off, -1)
    if kind == "zero":
        return np.zeros((n, n))
    return rotate(np.logspace(-14, 0, n) * np.sign(rng.standard_normal(n)))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 100, 144, 256])
@pytest.mark.parametrize("kind", ["random", "pm_pairs", "degenerate", "diagonal", "tridiagonal",
                                  "zero", "scaled"])
def test_eigenvalues_match_lapack(lib, n, kind):
    rng = np.random.default_rng(7 * n + len(kind))
    A = _case(rng, n, kind)
    got = _call(lib, "eig", A)
    ref = np.linalg.eigvalsh(A)
    scale = max(np.abs(ref).max(), 1.0 if kind == "zero" else 1e-300)
    assert np.abs(got - ref).max() <= 1e-13 * scale


def test_normalized_spectrum_of_a_paired_corner(lib):
    """|eigenvalues| in decreasing order over the largest: the pairs of a
    corner with a +-lambda spectrum come out as equal neighbours."""
    rng = np.random.default_rng(11)
    lam = np.sort(np.abs(rng.standard_normal(72)))[::-1]
    Q, _ = np.linalg.qr(rng.standard_normal((144, 144)))
    C = (Q * np.concatenate([lam, -lam])) @ Q.T
    s = _call(lib, "spec", (C + C.T) / 2)
    ref = np.repeat(lam, 2) / lam[0]
    assert abs(s[0] - 1.0) < 1e-14
    assert np.abs(s - ref).max() < 1e-13
