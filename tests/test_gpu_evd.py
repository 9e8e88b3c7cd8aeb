"""GPU eigendecomposition projector (the conventional CTMRG baseline, Fig.
3c) through the C interface: the eigensolver against LAPACK on matrices of
known spectrum, EVD-based CTMRG steps against the oracle's EVD variant, and
the D=4, chi=64 Kitaev workload against the stored oracle run."""
import json
import os

import numpy as np
import pytest
import torch

import ctm_inputs as ci
from oracle import ctm as oracle
from paper_2509_05090_amd import ctm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def known_spectrum_matrix(n, seed, lam):
    U, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return (U * lam) @ U.T


@pytest.mark.parametrize("n,k,kind", [(50, 10, "pm"), (300, 64, "gauss"), (1024, 64, "pm"),
                                      (129, 129, "gauss"), (2, 1, "gauss"), (1, 1, "gauss")])
def test_eigh_top_matches_lapack(n, k, kind):
    rng = np.random.default_rng(n + k)
    if kind == "pm":      # +-lambda pairs, as the enlarged corners of the workloads have
        half = rng.uniform(0.01, 1.0, (n + 1) // 2)
        lam = np.concatenate([half, -half])[:n] * (1 + 1e-3 * rng.standard_normal(n))
        A = known_spectrum_matrix(n, n, lam)
    else:
        A = rng.standard_normal((n, n))
        A = A + A.T
    U, w = ctm.eigh_top(torch.tensor(A, device=DEV), k)
    U = U.cpu().numpy()
    lam_ref, V = np.linalg.eigh(A)
    order = oracle.order_by_magnitude(lam_ref)[:k]
    scale = np.abs(lam_ref).max()
    assert np.abs(w - lam_ref[order]).max() < 1e-12 * scale
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    assert np.abs(A @ U - U * w).max() < 1e-11 * scale
    # largest entry of every column positive
    rows = np.argmax(np.abs(U), axis=0)
    assert (U[rows, np.arange(k)] > 0).all()


@pytest.mark.parametrize("D,chi,steps", [(2, 7, 4), (2, 16, 6), (3, 20, 3)])
def test_evd_steps_match_oracle(D, chi, steps):
    """Growth, first truncation and truncated steps with the eigendecomposition
    projector: corner spectrum and bond density matrix to rounding."""
    w = ci.Workload("t", 2, D, chi, 100 + D, 200 + chi)
    A = oracle.prepare_site_tensor(ci.raw_site_tensor(w))
    st = oracle.State(A, chi, ci.start_matrix(w), proj="evd")
    st.run(steps=steps)
    Ad = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(w), device=DEV))
    with ctm.Context(Ad, torch.tensor(ci.start_matrix(w), device=DEV), chi, proj="evd") as c:
        c.step(steps)
        s = c.spectrum()
        _, rho = c.energy(ci.heisenberg_rotated())
        C, T, _ = c.get_env()
    assert np.abs(s - st.spectrum).max() < 1e-10
    assert np.abs(rho - st.bond_density_matrix()).max() < 1e-11
    assert np.abs(C.cpu().numpy() - st.C).max() < 1e-8


def test_c2_evd_workload_matches_oracle():
    """D=4, chi=64 Kitaev workload to convergence with the eigendecomposition
    projector; energy and spectrum against the oracle's stored EVD run, and
    the QR projector's converged energy (the shared fixed point)."""
    wl = ci.WORKLOADS["c2"]
    gold = json.load(open(os.path.join(GOLDEN, "c2_evd.json")))
    A = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(wl), device=DEV))
    G = torch.tensor(ci.start_matrix(wl), device=DEV)
    with ctm.Context(A, G, wl.chi, proj="evd") as c:
        steps, delta, ok = c.converge(wl.tol, 400, n_check=1)
        e, _ = c.energy(ci.site_energy_operator(wl))
        s = c.spectrum()
    print(f"EVD: {steps} steps, delta {delta:.2e}, e {e:.15f}, oracle {gold['e_site']:.15f}")
    assert ok
    assert abs(e - gold["e_site"]) < 1e-10
    assert np.abs(s - np.array(gold["spectrum"])).max() < 1e-9
