"""FP64 CPU oracle of C3v-symmetric CTMRG on the honeycomb lattice.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg call it.  It shares no code with the HIP library.

Plain NumPy float64, written to be read against the paper (arXiv 2509.05090,
Yang & Corboz): Sec. II.A (double layer, local mapping of a 60-degree sector
onto a square quadrant, Fig. 1), Sec. II.B (corner and edge update rules and
the two projector constructions, Fig. 3), Sec. II.C (local expectation
values, Fig. 4b), Sec. III.A-B (Hamiltonian, sublattice rotation) and
Appendix A (C3v projection of the site tensor).

Tensor conventions (the figures are not available; the reading below is the
one pinned by the brute-force patch contraction in ``oracle/patch.py``):

* A[s, u, v, w]            site tensor, physical s, virtual u, v, w.
* a[I, J, K]               double layer, I = u*D + u' (ket index major).
* pair b[i, j, k, l] = sum_m a[i, j, m] a[m, k, l]: outer site legs i (+x),
  j (+y), inner site legs k (-y), l (-x); m is the pair's internal bond.
* C[gamma, delta]          corner, chi_c x chi_c, real symmetric.
* T[alpha, i, gamma]       edge: outer leg, end leg (towards the apex), inner
  leg (towards the corner).
* enlarged corner Ct[(alpha,k),(beta,l)] = sum T[alpha,i,gamma] C[gamma,delta]
  T[beta,j,delta] a[i,j,m] a[m,k,l], an n x n matrix with n = chi_c D^2.
"""
from __future__ import annotations

import itertools

import numpy as np

# ------------------------------------------------------------ Appendix A


def symmetrize(A: np.ndarray) -> np.ndarray:
    """C3v projection for the trivial irrep (U_g = 1, real tensor): the group
    average of Appendix A reduces to the mean over the 6 permutations of the
    three virtual legs (rotations permute cyclically, mirrors swap two legs;
    for a real tensor the complex conjugation of the anti-unitary mirrors is
    the identity)."""
    out = np.zeros_like(A)
    for p in itertools.permutations((1, 2, 3)):
        out += np.transpose(A, (0,) + p)
    return out / 6.0


def prepare_site_tensor(raw: np.ndarray) -> np.ndarray:
    """Project onto the symmetric subspace and normalize to unit Frobenius norm."""
    A = symmetrize(raw)
    return A / np.linalg.norm(A)


# ------------------------------------------------------------ Sec. II.A


def double_layer(A: np.ndarray) -> np.ndarray:
    """a = sum_s A[s,...] A*[s,...] (Fig. 1b); each leg fuses a ket index u and
    a bra index u' into I = u*D + u'.  A is real here, so A* = A."""
    D = A.shape[1]
    a = np.einsum("suvw,sxyz->uxvywz", A, A)
    return a.reshape(D * D, D * D, D * D)


def double_layer_open(A: np.ndarray) -> np.ndarray:
    """Double layer with the physical legs left open: a_O[I,J,K,s,s']."""
    D = A.shape[1]
    d = A.shape[0]
    ao = np.einsum("suvw,txyz->uxvywzst", A, A)
    return ao.reshape(D * D, D * D, D * D, d, d)


def initial_environment(D: int):
    """Small start (Sec. II.B): a 1x1 corner and an edge that closes the two
    layers of its single D^2 leg (ket and bra identified): T[0,(u,u'),0] =
    delta_{u u'}."""
    C = np.ones((1, 1))
    T = np.eye(D).reshape(1, D * D, 1)
    return C, T


# ------------------------------------------------------------ Sec. II.B, Fig. 3


def enlarged_corner(C: np.ndarray, T: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Ct = b . T . C . T (Fig. 3a,c): the new pair at the apex, the row edge
    on its +x leg, the column edge on its +y leg, the old corner between the
    two edges.  Returns the n x n matrix with rows (alpha, k), columns
    (beta, l)."""
    chi = C.shape[0]
    D2 = a.shape[0]
    CT = np.einsum("gd,bjd->gjb", C, T)                    # C on the column edge
    TCT = np.tensordot(T, CT, axes=([2], [0]))             # [alpha,i,j,beta]
    X = np.einsum("aijb,ijm->abm", TCT, a, optimize=True)  # outer site of the pair
    Ct = np.einsum("abm,mkl->akbl", X, a, optimize=True)   # inner site of the pair
    return Ct.reshape(chi * D2, chi * D2)


def gram_schmidt_basis(G: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of G with the unique sign choice
    diag(R) > 0, i.e. the Gram-Schmidt orthonormalization of G."""
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def align_signs(Q: np.ndarray, P_prev: np.ndarray) -> np.ndarray:
    """Column-sign gauge: flip column j when its overlap with the previous
    projector's column j is negative (zero overlap counts as positive)."""
    s = np.sign(np.sum(P_prev * Q, axis=0))
    s[s == 0] = 1.0
    return Q * s


def order_by_magnitude(lam: np.ndarray) -> np.ndarray:
    """Order eigenvalues by decreasing |lambda|, ties by larger signed
    lambda, then by lower index."""
    idx = np.arange(lam.size)
    return np.lexsort((idx, -lam, -np.abs(lam)))


def align_basis(Q: np.ndarray, P_prev: np.ndarray) -> np.ndarray:
    """Basis of span(Q) tied to the previous projector: the Gram-Schmidt
    orthonormalization (within span(Q)) of the projections of P_prev's
    columns, Q <- Q gs(Q^T P_prev).  If span(Q) = span(P_prev) this returns
    P_prev itself, so a converged projector is stationary element by
    element; the column overlaps Q^T P_prev come out upper triangular with a
    positive diagonal, which fixes the column signs as well."""
    return Q @ gram_schmidt_basis(Q.T @ P_prev)


def qr_projector(Ct, chi, P_prev, G, rr_gauge=False, gauge="align"):
    """QR-based projector (Fig. 3d).  The reduced corner is M = Ct P_prev, an
    n x chi matrix (chi D^2 x chi); its thin QR factor Q is the isometry.

    Reading of the unpublished network (the figure is missing): one sweep of
    orthogonal (subspace) iteration per CTMRG step.  At a fixed point
    Ct Q = Q R with Q^T Ct Q = R symmetric and triangular, hence diagonal, so
    Q spans a dominant eigenspace of Ct and the method shares the fixed point
    of the eigendecomposition-based CTMRG (Fig. 3c).

    The paper fixes no basis inside span(Q).  A QR factor alone does not
    converge element by element when Ct has eigenvalue pairs of equal
    modulus (for a pair +-lambda one QR sweep maps the 2x2 block
    [[a, b], [b, -a]] to [[a, -b], [-b, -a]], a two-cycle), and then P_prev no
    longer matches the basis of the next enlarged corner.  gauge="align"
    (default) ties the basis to P_prev with align_basis(); gauge="sign" only
    flips column signs to follow P_prev; rr_gauge adds a Rayleigh-Ritz
    rotation to the eigenbasis of Q^T Ct Q before the gauge step.

    Returns (Q, new P_prev)."""
    n = Ct.shape[0]
    if n <= chi:
        return np.eye(n), P_prev
    if P_prev is None or P_prev.shape != (n, chi):
        P_prev = gram_schmidt_basis(G[:n, :chi])
    M = Ct @ P_prev
    Q, _R = np.linalg.qr(M)
    if rr_gauge:
        w, V = np.linalg.eigh(Q.T @ Ct @ Q)
        Q = Q @ V[:, order_by_magnitude(w)]
    if gauge == "align":
        Q = align_basis(Q, P_prev)
    elif gauge == "sign":
        Q = align_signs(Q, P_prev)
    else:
        raise ValueError(gauge)
    return Q, Q


def evd_projector(Ct, chi, P_prev):
    """Conventional projector (Fig. 3c): eigenvectors of the Hermitian
    enlarged corner belonging to the chi largest |eigenvalues|.
    Returns (Q, new P_prev)."""
    n = Ct.shape[0]
    if n <= chi:
        return np.eye(n), P_prev
    lam, U = np.linalg.eigh(Ct)
    Q = U[:, order_by_magnitude(lam)[:chi]]
    if P_prev is not None and P_prev.shape == Q.shape:
        Q = align_signs(Q, P_prev)
    else:
        rows = np.argmax(np.abs(Q), axis=0)
        s = np.sign(Q[rows, np.arange(Q.shape[1])])
        s[s == 0] = 1.0
        Q = Q * s
    return Q, Q


def renormalize_corner(Ct, Q):
    """C' = P^dag Ct P (Fig. 3a), symmetrized and Frobenius-normalized."""
    C = Q.T @ Ct @ Q
    C = 0.5 * (C + C.T)
    return C / np.linalg.norm(C)


def renormalize_edge(T, a, Q):
    """T' = P^dag (T b) P (Fig. 3b): the new pair's +x leg joins the edge's
    end leg; its -y leg joins the outer side, its +y leg the inner side, and
    its -x leg becomes the new end leg.  Frobenius-normalized."""
    chi_c = T.shape[0]
    D2 = a.shape[0]
    Qr = Q.reshape(chi_c, D2, Q.shape[1])                     # [alpha,k,mu]
    V = np.einsum("aig,ijm->agjm", T, a, optimize=True)       # outer site
    V2 = np.einsum("agjm,gjn->amn", V, Qr, optimize=True)     # inner-side projector
    V3 = np.einsum("amn,mkl->ankl", V2, a, optimize=True)     # inner site
    Tn = np.einsum("akp,ankl->pln", Qr, V3, optimize=True)    # outer-side projector
    return Tn / np.linalg.norm(Tn)


def corner_spectrum(C):
    """Gauge-invariant convergence measure: |eigenvalues| of C in decreasing
    order, divided by the largest."""
    s = np.sort(np.abs(np.linalg.eigvalsh(C)))[::-1]
    return s / s[0]


def spectrum_change(s, s_prev):
    if s_prev is None:
        return np.inf
    m = max(s.size, s_prev.size)
    a = np.zeros(m)
    b = np.zeros(m)
    a[: s.size] = s
    b[: s_prev.size] = s_prev
    return float(np.max(np.abs(a - b)))


class State:
    """Environment of one CTMRG run."""

    def __init__(self, A, chi, G, proj="qr", rr_gauge=False, gauge="align"):
        self.A = np.asarray(A, dtype=np.float64)
        self.d, self.D = A.shape[0], A.shape[1]
        self.chi = chi
        self.G = G
        self.proj = proj
        self.rr_gauge = rr_gauge
        self.gauge = gauge
        self.a = double_layer(self.A)
        self.C, self.T = initial_environment(self.D)
        self.P = None
        self.spectrum = None
        self.steps = 0

    def projector(self, Ct, P_prev):
        if self.proj == "qr":
            return qr_projector(Ct, self.chi, P_prev, self.G, self.rr_gauge, self.gauge)
        if self.proj == "evd":
            return evd_projector(Ct, self.chi, P_prev)
        raise ValueError(self.proj)

    def step(self):
        """One CTMRG iteration; returns the corner-spectrum change."""
        Ct = enlarged_corner(self.C, self.T, self.a)
        Q, self.P = self.projector(Ct, self.P)
        Cn = renormalize_corner(Ct, Q)
        Tn = renormalize_edge(self.T, self.a, Q)
        self.C, self.T = Cn, Tn
        self.steps += 1
        s = corner_spectrum(self.C)
        delta = spectrum_change(s, self.spectrum)
        self.spectrum = s
        return delta

    def run(self, steps=None, tol=None, max_steps=10_000):
        """Fixed step count, or iterate until the spectrum change < tol."""
        delta = np.inf
        if steps is not None:
            for _ in range(steps):
                delta = self.step()
            return delta
        for _ in range(max_steps):
            delta = self.step()
            if delta < tol:
                break
        return delta

    # ---------------------------------------------------- Sec. II.C, Fig. 4b
    def measurement_environment(self):
        """Enlarged corner Ct of the current environment, a projector Q_m
        built by the run's own rule (the state is left unchanged), and the
        environment seen by one corner of the six-corner ring:
        Env = Q_m (Q_m^T Ct Q_m)^5 Q_m^T (Env = Ct^5 when nothing is cut)."""
        Ct = enlarged_corner(self.C, self.T, self.a)
        Q, _ = self.projector(Ct, self.P)
        Cr = Q.T @ Ct @ Q
        Cr = Cr / np.abs(Cr).max()
        Env = Q @ np.linalg.matrix_power(Cr, 5) @ Q.T
        return Env

    def bond_density_matrix(self):
        """rho[(s,t),(s',t')] of the apex pair of one sector (outer site s,
        inner site t), from the ring Tr(Ct_O Env); normalized to trace 1."""
        return bond_density_matrix(self.C, self.T, self.A, self.measurement_environment())

    def energy(self, h):
        return expectation(self.bond_density_matrix(), h)


def bond_density_matrix(C, T, A, Env):
    """rho = sum T C T a_O a_O Env: the enlarged corner with the apex pair's
    physical legs open, traced against the rest of the ring."""
    d = A.shape[0]
    ao = double_layer_open(A)                                   # [I,J,M,s,s']
    CT = np.einsum("gd,bjd->gjb", C, T)
    TCT = np.tensordot(T, CT, axes=([2], [0]))                  # [a,i,j,b]
    XO = np.einsum("aijb,ijmsu->abmsu", TCT, ao, optimize=True)  # outer site open
    chi = C.shape[0]
    D2 = ao.shape[0]
    Envr = Env.reshape(chi, D2, chi, D2)                        # [(b,l),(a,k)]
    EO = np.einsum("mklvw,blak->abmvw", ao, Envr, optimize=True)  # inner site open
    rho = np.einsum("abmsu,abmtw->stuw", XO, EO, optimize=True)  # [s,t,s',t']
    rho = rho.reshape(d * d, d * d)
    return rho / np.trace(rho)


def expectation(rho, h):
    """<O> = Tr(rho O) / Tr(rho) (Sec. II.C)."""
    return float(np.trace(rho @ h) / np.trace(rho))
