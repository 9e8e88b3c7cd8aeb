"""Pins of the oracle's reference gradient (no GPU): central finite
differences of converged energies, scale invariance, the symmetric subspace,
a D=1 analytic derivative, and convergence in the number of tracked steps."""
import math

import numpy as np
import pytest

import ctm_inputs as ci
from oracle import ctm, grad

H_SITE = 1.5 * ci.heisenberg_rotated()


def converged(A, chi, G, steps=400):
    st = ctm.State(A, chi, G, proj="qr")
    st.run(steps=steps)
    return st


@pytest.fixture(scope="module")
def setup():
    A = ctm.prepare_site_tensor(ci.gaussian((2, 2, 2, 2), 7))
    chi = 8
    G = ci.gaussian((chi * 4, chi), 99)
    st = converged(A, chi, G)
    E, g = grad.gradient(A, st.C, st.T, st.P, chi, 40, H_SITE)
    return A, chi, G, st, E, g


def test_gradient_matches_finite_differences(setup):
    A, chi, G, st, E, g = setup
    h = 1e-6
    for seed in (1100, 1101, 1102):
        v = ctm.symmetrize(ci.gaussian(A.shape, seed))
        v /= np.linalg.norm(v)
        Ep = converged(A + h * v, chi, G).energy(H_SITE)
        Em = converged(A - h * v, chi, G).energy(H_SITE)
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - np.sum(g * v)) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_scale_invariance_and_symmetry(setup):
    A, chi, G, st, E, g = setup
    assert abs(E - st.energy(H_SITE)) < 1e-13
    assert abs(np.sum(g * A)) < 1e-12
    assert np.allclose(ctm.symmetrize(g), g, atol=1e-15)


def test_tracked_steps_converge(setup):
    A, chi, G, st, E, g = setup
    _, g10 = grad.gradient(A, st.C, st.T, st.P, chi, 10, H_SITE)
    _, g80 = grad.gradient(A, st.C, st.T, st.P, chi, 80, H_SITE)
    assert np.abs(g80 - g).max() <= np.abs(g10 - g).max() + 1e-13
    assert np.abs(g80 - g).max() < 1e-10


def test_torch_twin_matches_numpy_forward(setup):
    A, chi, G, st, E, g = setup
    import torch
    rho_t = grad.bond_density_matrix(torch.tensor(st.C), torch.tensor(st.T),
                                     torch.tensor(A), torch.tensor(st.P), chi)
    assert np.abs(rho_t.numpy() - st.bond_density_matrix()).max() < 1e-14


@pytest.mark.parametrize("theta", [0.3, 1.2])
def test_product_state_analytic_gradient(theta):
    """D=1: <SzSz> = m^2 with m = (p0^2 - p1^2) / (2 (p0^2 + p1^2)); its
    derivative in (p0, p1) written out by hand."""
    p0, p1 = math.cos(theta) * 1.3, math.sin(theta) * 1.3
    A = np.array([p0, p1]).reshape(2, 1, 1, 1)
    st = ctm.State(A, 4, None)
    st.run(steps=2)
    E, g = grad.gradient(A, st.C, st.T, st.P, 4, 2, ci.szsz())
    N = p0 ** 2 + p1 ** 2
    m = (p0 ** 2 - p1 ** 2) / (2 * N)
    ref = np.array([2 * m * 2 * p0 * p1 ** 2 / N ** 2, -2 * m * 2 * p1 * p0 ** 2 / N ** 2])
    assert abs(E - m * m) < 1e-14
    assert np.abs(g.reshape(2) - ref).max() < 1e-13
