"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each check ties the oracle to something it does not compute itself: closed
forms of product states, brute-force contraction of finite honeycomb
patches built from coordinates, exact invariants (symmetry, isometry,
Hermiticity, gauge invariance), the shared fixed point of the QR and
eigendecomposition projectors, and finite differences of the energy.
"""
import itertools
import math

import numpy as np
import pytest

import ctm_inputs as ci
from oracle import ctm, patch

H_ROT = ci.heisenberg_rotated()


def rand_sym(d, D, seed):
    return ctm.prepare_site_tensor(ci.gaussian((d, D, D, D), seed))


# ------------------------------------------------------------------ P9
def test_symmetrizer_is_orthogonal_projector():
    x = ci.gaussian((2, 3, 3, 3), 1)
    y = ci.gaussian((2, 3, 3, 3), 2)
    sx = ctm.symmetrize(x)
    assert np.allclose(ctm.symmetrize(sx), sx, atol=1e-15)
    assert abs(np.sum(sx * y) - np.sum(x * ctm.symmetrize(y))) < 1e-13
    for p in itertools.permutations((1, 2, 3)):
        assert np.array_equal(np.transpose(sx, (0,) + p), sx) or \
            np.allclose(np.transpose(sx, (0,) + p), sx, atol=1e-15)
    # a generic tensor is not symmetric
    assert np.linalg.norm(sx - x) > 0.1


def test_symmetrizer_matches_explicit_group_average():
    """The six C3v elements act on the virtual legs (u, v, w) as the three
    cyclic rotations and three two-leg swaps; written out by hand."""
    x = ci.gaussian((2, 2, 2, 2), 3)
    perms = [(1, 2, 3), (2, 3, 1), (3, 1, 2), (2, 1, 3), (1, 3, 2), (3, 2, 1)]
    ref = sum(np.transpose(x, (0,) + p) for p in perms) / 6
    assert np.allclose(ctm.symmetrize(x), ref, atol=1e-15)


def test_double_layer_fully_symmetric():
    A = rand_sym(2, 3, 4)
    a = ctm.double_layer(A)
    for p in itertools.permutations((0, 1, 2)):
        assert np.allclose(np.transpose(a, p), a, atol=1e-15)
    # a[(u,u'),(v,v'),(w,w')] = sum_s A[s,u,v,w] A[s,u',v',w'] entry by entry
    D = 3
    for (u, up, v, vp, w, wp) in [(0, 1, 2, 0, 1, 1), (2, 2, 0, 1, 0, 2)]:
        ref = sum(A[s, u, v, w] * A[s, up, vp, wp] for s in range(2))
        assert abs(a[u * D + up, v * D + vp, w * D + wp] - ref) < 1e-15


# ------------------------------------------------------------------ P1, P2
def product_state(theta, D=1):
    A = np.zeros((2, D, D, D))
    A[0, 0, 0, 0] = math.cos(theta)
    A[1, 0, 0, 0] = math.sin(theta)
    return A


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, 2.5])
def test_product_state_closed_forms_D1(theta):
    A = product_state(theta)
    st = ctm.State(A, 4, None)
    assert st.run(steps=3) < 1e-15
    assert st.C.shape == (1, 1) and np.allclose(st.spectrum, [1.0])
    rho = st.bond_density_matrix()
    # rotated Heisenberg: E_site = -3J/8 for every real product state
    assert abs(1.5 * ctm.expectation(rho, H_ROT) + 3 / 8) < 1e-14
    # Sz Sz: <Sz>^2 = cos^2(2 theta) / 4
    assert abs(ctm.expectation(rho, ci.szsz()) - math.cos(2 * theta) ** 2 / 4) < 1e-14
    # Kitaev-Heisenberg, unrotated: E_site = (K + 3J)/8
    K, J = math.cos(ci.KH_PHI), math.sin(ci.KH_PHI)
    e = 0.5 * sum(ctm.expectation(rho, ci.kh_bond(al, K, J)) for al in "xyz")
    assert abs(e - (K + 3 * J) / 8) < 1e-14
    assert abs((K + 3 * J) / 8 - 0.3768545) < 1e-6


@pytest.mark.parametrize("D,chi,proj", [(2, 2, "qr"), (2, 3, "evd"), (4, 5, "qr"), (2, 16, "qr")])
def test_product_state_embedded(D, chi, proj):
    """The D=1 product state embedded in a larger bond space goes through the
    growth and truncation paths and must give the same closed forms."""
    theta = 0.7
    A = product_state(theta, D)
    G = ci.gaussian((chi * D * D, chi), 5)
    st = ctm.State(A, chi, G, proj=proj)
    st.run(steps=6)
    rho = st.bond_density_matrix()
    assert abs(1.5 * ctm.expectation(rho, H_ROT) + 3 / 8) < 1e-13
    assert abs(ctm.expectation(rho, ci.szsz()) - math.cos(2 * theta) ** 2 / 4) < 1e-13


# ------------------------------------------------------------------ P3, P11
def test_patch_is_a_honeycomb_piece():
    """The six sectors give 12 N^2 distinct honeycomb sites, every site has at
    most 3 neighbours, and every honeycomb site within distance 1.5 N of the
    hexagon centre belongs to the patch."""
    N = 3
    pts, outer0, inner0 = patch.patch_sites(N)
    assert len(pts) == 12 * N * N
    dist = np.linalg.norm(pts[:, None] - pts[None], axis=-1)
    assert dist[np.triu_indices(len(pts), 1)].min() > 0.99
    assert ((np.abs(dist - 1) < 1e-9).sum(1) <= 3).all()
    # all honeycomb sites (pointy-top, hexagon centre at 0) near the origin
    s3 = math.sqrt(3)
    a1, a2 = np.array([s3, 0]), np.array([s3 / 2, 1.5])
    lat = []
    for i in range(-10, 11):
        for j in range(-10, 11):
            c = i * a1 + j * a2
            for k in range(6):
                t = math.pi / 6 + math.pi / 3 * k
                lat.append(c + np.array([math.cos(t), math.sin(t)]))
    lat = np.unique(np.round(np.array(lat), 9), axis=0)
    near = lat[np.linalg.norm(lat, axis=1) <= 1.5 * N]
    for q in near:
        assert np.linalg.norm(pts - q, axis=1).min() < 1e-9
    assert np.allclose(pts[outer0], [0, 2]) and np.allclose(pts[inner0], [0, 1])


@pytest.mark.parametrize("D,N,seed", [(2, 1, 7), (2, 2, 7), (2, 3, 8), (3, 1, 9), (3, 2, 10)])
def test_ring_equals_brute_force_patch(D, N, seed):
    """N-1 untruncated steps, then the six-corner ring with the apex pair
    open, must equal the direct contraction of the 12 N^2-site patch."""
    A = rand_sym(2, D, seed)
    st = ctm.State(A, 10 ** 9, None)
    for _ in range(N - 1):
        st.step()
    assert np.allclose(st.bond_density_matrix(), patch.patch_density_matrix(A, N),
                       atol=1e-13, rtol=0)


def test_ring_partition_function():
    A = rand_sym(2, 2, 11)
    st = ctm.State(A, 10 ** 9, None)
    Ct = ctm.enlarged_corner(st.C, st.T, st.a)
    z = np.trace(np.linalg.matrix_power(Ct, 6))
    assert abs(z - patch.patch_norm(A, 1)) < 1e-13 * abs(z)


def test_brute_force_catches_transposed_edge(monkeypatch):
    """A planted mistake in the edge update (inner and outer legs of the new
    pair swapped) must be caught by the patch comparison."""
    A = rand_sym(2, 2, 12)
    good = patch.patch_density_matrix(A, 3)

    orig = ctm.renormalize_edge

    def bad_edge(T, a, Q):
        return np.ascontiguousarray(np.transpose(orig(T, a, Q), (2, 1, 0)))  # outer <-> inner

    monkeypatch.setattr(ctm, "renormalize_edge", bad_edge)
    st = ctm.State(A, 10 ** 9, None)
    st.step()
    st.step()
    assert np.abs(st.bond_density_matrix() - good).max() > 1e-6


def test_brute_force_catches_wrong_corner(monkeypatch):
    A = rand_sym(2, 2, 13)
    good = patch.patch_density_matrix(A, 2)
    orig = ctm.enlarged_corner

    def bad_corner(C, T, a):
        return orig(C, np.transpose(T, (2, 1, 0)).copy(), a)   # edge legs swapped

    monkeypatch.setattr(ctm, "enlarged_corner", bad_corner)
    st = ctm.State(A, 10 ** 9, None)
    st.step()
    assert np.abs(st.bond_density_matrix() - good).max() > 1e-6


# ------------------------------------------------------------------ P4, P5
def truncated_state(D=2, chi=8, steps=30, proj="qr", seed=7, rr=False, gauge="align"):
    A = rand_sym(2, D, seed)
    G = ci.gaussian((chi * D * D, chi), 99)
    st = ctm.State(A, chi, G, proj=proj, rr_gauge=rr, gauge="sign" if rr else gauge)
    st.run(steps=steps)
    return st


def test_enlarged_corner_hermitian_and_isometry():
    st = truncated_state(D=3, chi=12, steps=8)
    Ct = ctm.enlarged_corner(st.C, st.T, st.a)
    assert np.abs(Ct - Ct.T).max() <= 1e-14 * np.abs(Ct).max()
    Q, _ = ctm.qr_projector(Ct, st.chi, st.P, st.G)
    assert Q.shape == (Ct.shape[0], st.chi)
    assert np.abs(Q.T @ Q - np.eye(st.chi)).max() < 1e-13
    C = Q.T @ Ct @ Q
    assert np.abs(C - C.T).max() <= 1e-13 * np.abs(C).max()
    Qe, _ = ctm.evd_projector(Ct, st.chi, None)
    assert np.abs(Qe.T @ Qe - np.eye(st.chi)).max() < 1e-13


def test_gram_schmidt_basis_is_classical_gram_schmidt():
    G = ci.gaussian((20, 5), 21)
    Q = ctm.gram_schmidt_basis(G)
    ref = np.zeros_like(G)
    for j in range(G.shape[1]):
        v = G[:, j].copy()
        for i in range(j):
            v -= (ref[:, i] @ G[:, j]) * ref[:, i]
        ref[:, j] = v / np.linalg.norm(v)
    assert np.allclose(Q, ref, atol=1e-12)


def test_evd_projector_keeps_largest_magnitudes():
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    lam = np.array([5.0, -4.0, 4.0, -3.0, 2.5, -0.1, 0.05, 1.0, -1.5, 0.0])
    M = (U * lam) @ U.T
    Q, _ = ctm.evd_projector(M, 4, None)
    w = np.sort(np.linalg.eigvalsh(Q.T @ M @ Q))
    assert np.allclose(w, np.sort([5.0, 4.0, -4.0, -3.0]), atol=1e-12)
    # ties in |lambda|: larger signed value first
    assert list(ctm.order_by_magnitude(np.array([-2.0, 2.0, 1.0, -3.0]))) == [3, 1, 0, 2]


# ------------------------------------------------------------------ P6, P7
def test_qr_and_evd_share_the_fixed_point():
    """Same site tensor and chi: the QR (subspace-iteration) projector and the
    eigendecomposition projector converge to the same spectrum and energy."""
    out = {}
    for proj in ("qr", "evd"):
        st = truncated_state(D=2, chi=8, steps=400, proj=proj)
        out[proj] = (st.energy(H_ROT), st.spectrum)
    assert abs(out["qr"][0] - out["evd"][0]) < 1e-12
    assert np.abs(out["qr"][1] - out["evd"][1]).max() < 1e-10
    # the value the independent survey scripts printed for this input (seed 7)
    assert abs(1.5 * out["qr"][0] - (-0.37503455941553)) < 1e-13


def test_rayleigh_ritz_gives_elementwise_fixed_point():
    st = truncated_state(D=2, chi=8, steps=300, rr=True)
    C0, T0 = st.C.copy(), st.T.copy()
    st.step()
    assert np.abs(st.C - np.diag(np.diag(st.C))).max() < 1e-12
    assert np.abs(st.C - C0).max() < 1e-12
    assert np.abs(st.T - T0).max() < 1e-12
    Ct = ctm.enlarged_corner(st.C, st.T, st.a)
    Q = st.P
    lhs = Ct @ Q
    C = Q.T @ Ct @ Q
    assert np.linalg.norm(lhs - Q @ C) / np.linalg.norm(Ct) < 1e-10


def test_sign_gauge_two_cycle_on_plus_minus_pair():
    """Why the basis must be tied to P_prev: for an exact +-lambda pair one
    QR sweep flips the off-diagonal of the 2x2 block, a two-cycle that column
    signs cannot remove; the aligned basis is stationary."""
    a, b = 0.6, 0.8
    Ct = np.array([[a, b], [b, -a]])          # eigenvalues +-1
    P = np.eye(2)
    Q, _ = np.linalg.qr(Ct @ P)
    C1 = ctm.align_signs(Q, P).T @ Ct @ ctm.align_signs(Q, P)
    assert abs(C1[0, 1] + b) < 1e-15          # off-diagonal flipped
    Qa = ctm.align_basis(Q, P)
    assert np.abs(Qa - P).max() < 1e-15       # aligned basis: no change


def test_align_basis_properties():
    r = np.random.default_rng(3)
    Q, _ = np.linalg.qr(r.standard_normal((30, 6)))
    P, _ = np.linalg.qr(r.standard_normal((30, 6)))
    Qa = ctm.align_basis(Q, P)
    assert np.abs(Qa.T @ Qa - np.eye(6)).max() < 1e-14          # isometry
    assert np.abs(Qa @ Qa.T - Q @ Q.T).max() < 1e-14            # same span
    O = Qa.T @ P
    assert np.abs(np.tril(O, -1)).max() < 1e-14 and (np.diag(O) > 0).all()
    U, _ = np.linalg.qr(r.standard_normal((6, 6)))
    assert np.abs(ctm.align_basis(P @ U, P) - P).max() < 1e-14  # fixed point


def test_plus_minus_pairs_converge_to_evd_fixed_point():
    """Seed 1002 at D=4 gives an enlarged corner whose spectrum pairs as
    +-lambda; the aligned QR projector must still reach the energy of the
    eigendecomposition projector (chi=16)."""
    A = ctm.prepare_site_tensor(ci.gaussian((2, 4, 4, 4), 1002))
    G = ci.gaussian((16 * 16, 16), 1009)
    e = {}
    for proj in ("qr", "evd"):
        st = ctm.State(A, 16, G, proj=proj)
        st.run(steps=400 if proj == "qr" else 60)
        e[proj] = st.energy(H_ROT)
    lam = np.linalg.eigvalsh(ctm.enlarged_corner(st.C, st.T, st.a))
    lam = lam[ctm.order_by_magnitude(lam)]
    assert abs(abs(lam[0]) - abs(lam[1])) < 1e-10 * abs(lam[0]) and lam[0] * lam[1] < 0
    assert abs(e["qr"] - e["evd"]) < 1e-10


def test_subspace_residual_small_without_rr():
    st = truncated_state(D=2, chi=8, steps=400)
    Ct = ctm.enlarged_corner(st.C, st.T, st.a)
    Q = st.P
    C = Q.T @ Ct @ Q
    assert np.linalg.norm(Ct @ Q - Q @ C) / np.linalg.norm(Ct) < 1e-6


# ------------------------------------------------------------------ P8
def test_gauge_invariance_of_energy_and_spectrum():
    st = truncated_state(D=2, chi=8, steps=40)
    e0, s0 = st.energy(H_ROT), ctm.corner_spectrum(st.C)
    rng = np.random.default_rng(17)
    s = rng.choice([-1.0, 1.0], size=st.chi)
    st.C = (s[:, None] * st.C) * s[None, :]
    st.T = st.T * s[:, None, None] * s[None, None, :]
    # the next reduced corner Ct P_prev reads P_prev's rows (alpha, k) in the
    # current gauge of alpha
    st.P = st.P * np.repeat(s, st.D * st.D)[:, None]
    assert abs(st.energy(H_ROT) - e0) < 1e-14
    assert np.abs(ctm.corner_spectrum(st.C) - s0).max() < 1e-14


def test_spectrum_change_pads_with_zeros():
    assert ctm.spectrum_change(np.array([1.0, 0.5]), np.array([1.0])) == 0.5
    assert ctm.spectrum_change(np.array([1.0]), None) == np.inf
