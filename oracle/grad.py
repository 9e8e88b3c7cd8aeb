"""Reference energy gradient by automatic differentiation (torch, CPU, float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/ctm.py``).

The paper obtains dE/dA by differentiating through k tracked CTMRG steps
that follow untracked warm-up steps (Sec. II.D; k per bond dimension in
Tables I and II).  This module is a torch twin of the NumPy oracle's
corner, edge, projector and measurement steps, used only to get that
derivative: starting from a converged environment (detached), it runs k
differentiable steps and the bond-energy contraction, then back-propagates.
As k grows the result converges to the total derivative through the fixed
point, the quantity a fixed-point adjoint computes.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

DT = torch.float64


def symmetrize(A: torch.Tensor) -> torch.Tensor:
    """Trivial-irrep C3v projection: mean over the 6 virtual-leg permutations."""
    out = torch.zeros_like(A)
    for p in itertools.permutations((1, 2, 3)):
        out = out + A.permute((0,) + p)
    return out / 6.0


def double_layer(A):
    D = A.shape[1]
    return torch.einsum("suvw,sxyz->uxvywz", A, A).reshape(D * D, D * D, D * D)


def double_layer_open(A):
    D, d = A.shape[1], A.shape[0]
    return torch.einsum("suvw,txyz->uxvywzst", A, A).reshape(D * D, D * D, D * D, d, d)


def enlarged_corner(C, T, a):
    chi, D2 = C.shape[0], a.shape[0]
    CT = torch.einsum("gd,bjd->gjb", C, T)
    TCT = torch.tensordot(T, CT, dims=([2], [0]))
    X = torch.einsum("aijb,ijm->abm", TCT, a)
    Ct = torch.einsum("abm,mkl->akbl", X, a)
    return Ct.reshape(chi * D2, chi * D2)


def gram_schmidt_basis(G):
    """Orthonormal basis of G's columns with diag(R) > 0 (differentiable)."""
    Q, R = torch.linalg.qr(G)
    s = torch.sign(torch.diagonal(R)).detach()
    s[s == 0] = 1.0
    return Q * s


def qr_projector(Ct, chi, P_prev):
    """Q from the thin QR of the reduced corner Ct P_prev, its basis tied to
    P_prev by Q <- Q gs(Q^T P_prev) (the oracle's default gauge)."""
    n = Ct.shape[0]
    if n <= chi:
        return torch.eye(n, dtype=DT), P_prev
    Q, _ = torch.linalg.qr(Ct @ P_prev)
    Q = Q @ gram_schmidt_basis(Q.T @ P_prev)
    return Q, Q


def renormalize_corner(Ct, Q):
    C = Q.T @ Ct @ Q
    C = 0.5 * (C + C.T)
    return C / torch.linalg.norm(C)


def renormalize_edge(T, a, Q):
    chi_c, D2 = T.shape[0], a.shape[0]
    Qr = Q.reshape(chi_c, D2, Q.shape[1])
    V = torch.einsum("aig,ijm->agjm", T, a)
    V2 = torch.einsum("agjm,gjn->amn", V, Qr)
    V3 = torch.einsum("amn,mkl->ankl", V2, a)
    Tn = torch.einsum("akp,ankl->pln", Qr, V3)
    return Tn / torch.linalg.norm(Tn)


def bond_density_matrix(C, T, A, P_prev, chi):
    a = double_layer(A)
    Ct = enlarged_corner(C, T, a)
    Q, _ = qr_projector(Ct, chi, P_prev)
    Cr = Q.T @ Ct @ Q
    Cr = Cr / Cr.detach().abs().max()
    Env = Q @ torch.linalg.matrix_power(Cr, 5) @ Q.T
    ao = double_layer_open(A)
    d = A.shape[0]
    CT = torch.einsum("gd,bjd->gjb", C, T)
    TCT = torch.tensordot(T, CT, dims=([2], [0]))
    XO = torch.einsum("aijb,ijmsu->abmsu", TCT, ao)
    chi_c, D2 = C.shape[0], ao.shape[0]
    Envr = Env.reshape(chi_c, D2, chi_c, D2)
    EO = torch.einsum("mklvw,blak->abmvw", ao, Envr)
    rho = torch.einsum("abmsu,abmtw->stuw", XO, EO).reshape(d * d, d * d)
    return rho / torch.trace(rho)


def tracked_energy(A, C0, T0, P0, chi, k, h):
    """Tr(rho h) after k differentiable QR-CTMRG steps from (C0, T0, P0)."""
    a = double_layer(A)
    C, T, P = C0, T0, P0
    for _ in range(k):
        Ct = enlarged_corner(C, T, a)
        Q, P = qr_projector(Ct, chi, P)
        C, T = renormalize_corner(Ct, Q), renormalize_edge(T, a, Q)
    rho = bond_density_matrix(C, T, A, P, chi)
    return torch.trace(rho @ h)


def gradient(A: np.ndarray, C0, T0, P0, chi: int, k: int, h: np.ndarray):
    """(E, g): energy Tr(rho h) and g = sym(dE/dA) through k tracked steps
    from the given (detached) environment."""
    At = torch.tensor(A, dtype=DT, requires_grad=True)
    E = tracked_energy(At, torch.tensor(C0, dtype=DT), torch.tensor(T0, dtype=DT),
                       None if P0 is None else torch.tensor(P0, dtype=DT),
                       chi, k, torch.tensor(h, dtype=DT))
    (g,) = torch.autograd.grad(E, At)
    return float(E), symmetrize(g).numpy()
