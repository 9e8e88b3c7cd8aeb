"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds no CTMRG arithmetic.  It only draws the random numbers a
run needs and writes down the model Hamiltonians; both sides receive the same
arrays and do everything else on their own:

* raw site tensors: i.i.d. N(0,1) entries of shape (d, D, D, D), index order
  [s][u][v][w] (physical, then the three virtual legs).  Each side projects
  them onto the C3v-symmetric subspace and normalizes them itself;
* the start matrix G (chi*D^2 x chi, N(0,1)) whose orthonormal basis is the
  first QR projector (the paper does not say how the first projector is
  seeded; a seeded Gaussian is the reading used here);
* bond Hamiltonians of the Kitaev-Heisenberg model (Sec. III.A) on one
  nearest-neighbour bond, as d^2 x d^2 real matrices acting on
  (outer site, inner site), and the Heisenberg form after the pi-rotation
  about y on one sublattice (Sec. III.B).

Every generator is NumPy's PCG64 through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: shapes, seeds and the Hamiltonian it measures."""
    name: str
    d: int
    D: int
    chi: int
    seed_A: int
    seed_G: int
    seed_A2: int | None = None      # optional second tensor, added with weight eps
    eps: float = 0.0
    model: str = "heisenberg"       # heisenberg | kitaev | kh
    steps: int | None = None        # fixed step count, or None = to tolerance
    tol: float = 1e-12

    @property
    def D2(self) -> int:
        return self.D * self.D

    @property
    def n(self) -> int:
        return self.chi * self.D * self.D


# The five workloads: shapes inside the paper's own ranges (Sec. III.B, III.C).
WORKLOADS = {
    "c1": Workload("c1", 2, 2, 16, 1001, 1008, model="heisenberg", steps=50),
    "c2": Workload("c2", 2, 4, 64, 1002, 1009, model="kitaev", tol=1e-12),
    "c3": Workload("c3", 2, 6, 144, 1003, 1010, seed_A2=1004, eps=1e-2,
                   model="heisenberg", tol=1e-12),
    "c4": Workload("c4", 2, 4, 100, 1005, 1012, model="kh", tol=1e-12),
    "c5": Workload("c5", 2, 8, 256, 1006, 1013, model="heisenberg", tol=1e-8),
    # the shape of the paper's timing comparison of the two projectors (Sec. III.B)
    "p5": Workload("p5", 2, 5, 120, 1007, 1014, model="heisenberg", tol=1e-10),
}

KH_PHI = 0.3 * math.pi
DIRECTION_SEEDS = tuple(range(1100, 1120))


def raw_site_tensor(w: Workload) -> np.ndarray:
    """Unsymmetrized raw tensor R = G0 (+ eps * G1); float64, [s][u][v][w]."""
    shape = (w.d, w.D, w.D, w.D)
    r = np.random.default_rng(w.seed_A).standard_normal(shape)
    if w.seed_A2 is not None:
        r = r + w.eps * np.random.default_rng(w.seed_A2).standard_normal(shape)
    return np.ascontiguousarray(r, dtype=np.float64)


def gaussian(shape, seed: int) -> np.ndarray:
    return np.ascontiguousarray(
        np.random.default_rng(seed).standard_normal(shape), dtype=np.float64)


def start_matrix(w: Workload) -> np.ndarray:
    """Seeded N(0,1) matrix of shape (chi*D^2, chi); its first n rows seed
    the first projector of an n-row reduced corner."""
    return gaussian((w.n, w.chi), w.seed_G)


def direction(w: Workload, seed: int) -> np.ndarray:
    """Raw N(0,1) tangent direction for finite-difference checks."""
    return gaussian((w.d, w.D, w.D, w.D), seed)


# ---------------------------------------------------------------- operators
def spin_half():
    """S^x, S^y, S^z for spin 1/2 in the (up, down) basis; S^y is complex."""
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128) / 2
    sy = np.array([[0, -1j], [1j, 0]], dtype=np.complex128) / 2
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128) / 2
    return sx, sy, sz


def _real(m: np.ndarray) -> np.ndarray:
    assert np.abs(m.imag).max() < 1e-15
    return np.ascontiguousarray(m.real)


def heisenberg_rotated(J: float = 1.0) -> np.ndarray:
    """J S_i.S_j after a pi rotation about y on the inner site's sublattice:
    J (-SxSx + SySy - SzSz).  Acts on (outer, inner); 4x4 real."""
    sx, sy, sz = spin_half()
    h = J * (-np.kron(sx, sx) + np.kron(sy, sy) - np.kron(sz, sz))
    return _real(h)


def heisenberg(J: float = 1.0) -> np.ndarray:
    sx, sy, sz = spin_half()
    return _real(J * (np.kron(sx, sx) + np.kron(sy, sy) + np.kron(sz, sz)))


def kh_bond(alpha: str, K: float, J: float) -> np.ndarray:
    """K S^a S^a + J S.S on an alpha-bond (alpha in 'xyz'), unrotated."""
    sx, sy, sz = spin_half()
    s = {"x": sx, "y": sy, "z": sz}[alpha]
    return _real(K * np.kron(s, s)) + heisenberg(J)


def szsz() -> np.ndarray:
    sz = spin_half()[2]
    return _real(np.kron(sz, sz))


def bond_operators(w: Workload) -> dict:
    """Named bond operators measured for a workload.  The per-site energy is
    half the sum of the three bond energies (three bonds per site, each
    shared by two sites)."""
    if w.model == "heisenberg":
        h = heisenberg_rotated(1.0)
        return {"x": h, "y": h, "z": h}
    if w.model == "kitaev":
        return {a: kh_bond(a, 1.0, 0.0) for a in "xyz"}
    if w.model == "kh":
        K, J = math.cos(KH_PHI), math.sin(KH_PHI)
        return {a: kh_bond(a, K, J) for a in "xyz"}
    raise ValueError(w.model)


def site_energy_operator(w: Workload) -> np.ndarray:
    """(3/2) * mean of the three bond operators: with one bond density matrix
    shared by all bonds, Tr(rho h_site)/Tr(rho) is the energy per site."""
    ops = bond_operators(w)
    return 0.5 * (ops["x"] + ops["y"] + ops["z"])
