"""GPU parity of the CTMRG iteration against the CPU oracle, through the C
interface: identical seeded inputs, element-by-element comparison of the
environment (the column-sign gauge is fixed by the same rule on both
sides), corner spectra and bond energies."""
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


def gpu_context(w, prec="fp64"):
    raw = ci.raw_site_tensor(w)
    A = ctm.symmetrize(torch.tensor(raw, device=DEV))
    G = torch.tensor(ci.start_matrix(w), device=DEV)
    return ctm.Context(A, G, w.chi, prec=prec), A


def oracle_state(w, proj="qr"):
    A = oracle.prepare_site_tensor(ci.raw_site_tensor(w))
    return oracle.State(A, w.chi, ci.start_matrix(w), proj=proj)


def test_symmetrize_matches_oracle():
    for D in (1, 2, 3, 6, 8):
        raw = ci.gaussian((2, D, D, D), 40 + D)
        A = ctm.symmetrize(torch.tensor(raw, device=DEV)).cpu().numpy()
        assert np.abs(A - oracle.prepare_site_tensor(raw)).max() < 1e-15


def test_init_rejects_unsymmetric_tensor():
    w = ci.Workload("t", 2, 2, 8, 1, 2)
    raw = torch.tensor(ci.raw_site_tensor(w), device=DEV)
    G = torch.tensor(ci.start_matrix(w), device=DEV)
    with pytest.raises(ctm.CtmError) as ex:
        ctm.Context(raw, G, w.chi)
    assert ex.value.code == ctm.CTM_ENOTSYM


@pytest.mark.parametrize("D,chi,steps", [(2, 16, 1), (2, 16, 2), (2, 16, 3), (2, 16, 6), (2, 7, 5),
                                         (3, 20, 4)])
def test_steps_match_oracle(D, chi, steps):
    """Growth (n <= chi), first truncation, and truncated steps with ragged
    chi.  Gauge-invariant results (corner spectrum, bond density matrix) must
    agree to rounding.  C, T and the projector are compared element by
    element to 1e-8: the reduced corner M is badly conditioned right after
    the first truncation (cond(M) ~ 2e7 here), so two valid FP64 QRs differ
    by ~eps*cond(M) in the weak columns of Q1, the basis alignment spreads
    that over all columns, and the inherited basis keeps it."""
    w = ci.Workload("t", 2, D, chi, 100 + D, 200 + chi)
    c, _ = gpu_context(w)
    st = oracle_state(w)
    c.step(steps)
    st.run(steps=steps)
    C, T, P = c.get_env()
    torch.cuda.synchronize()
    assert C.shape == st.C.shape and T.shape == st.T.shape
    s = c.spectrum()
    assert np.abs(s - st.spectrum).max() < 1e-10
    _, rho = c.energy(ci.heisenberg_rotated())
    assert np.abs(rho - st.bond_density_matrix()).max() < 1e-11
    tol = 1e-12 if st.P is None else 1e-8
    assert np.abs(C.cpu().numpy() - st.C).max() < tol
    assert np.abs(T.cpu().numpy() - st.T).max() < tol
    if st.P is not None:
        assert np.abs(P.cpu().numpy() - st.P).max() < 1e-7
    c.close()


def test_c1_workload_energy_and_spectrum():
    """50 steps of QR-CTMRG at d=2, D=2, chi=16 (Heisenberg, FP64)."""
    w = ci.WORKLOADS["c1"]
    gold = json.load(open(os.path.join(GOLDEN, "c1_qr.json")))
    c, _ = gpu_context(w)
    c.step(w.steps)
    e, rho = c.energy(ci.heisenberg_rotated())
    s = c.spectrum()
    c.close()
    assert abs(e - gold["e_bond"]["x"]) < 1e-10
    assert np.abs(rho - np.array(gold["rho"])).max() < 1e-10
    assert np.abs(s - np.array(gold["spectrum"])).max() < 1e-10


def test_energy_untruncated_matches_oracle():
    """Energy evaluation in the growth regime (projector = identity)."""
    w = ci.Workload("t", 2, 2, 64, 301, 302)
    c, _ = gpu_context(w)
    st = oracle_state(w)
    for k in range(3):
        e, rho = c.energy(ci.heisenberg_rotated())
        assert np.abs(rho - st.bond_density_matrix()).max() < 1e-13
        c.step(1)
        st.step()
    c.close()


def _gold(name):
    return json.load(open(os.path.join(GOLDEN, name)))


@pytest.mark.parametrize("key", ["c2", "c4"])
def test_workload_fp64_matches_oracle(key):
    """Full workloads in FP64: the same number of steps as the stored oracle
    run; bond energies to 1e-10, corner spectrum to 1e-9."""
    w = ci.WORKLOADS[key]
    gold = _gold(f"{key}_qr.json")
    c, _ = gpu_context(w)
    c.step(gold["steps"])
    ops = ci.bond_operators(w)
    for name, h in ops.items():
        e, _ = c.energy(h)
        assert abs(e - gold["e_bond"][name]) < 1e-10, (name, e, gold["e_bond"][name])
    s = c.spectrum()
    assert np.abs(s - np.array(gold["spectrum"])).max() < 1e-9
    c.close()


def test_c2_qr_gpu_reaches_evd_oracle_energy():
    """QR-based CTMRG on the GPU and eigendecomposition-based CTMRG in the
    oracle converge to the same energy (the shared fixed point)."""
    w = ci.WORKLOADS["c2"]
    gold = _gold("c2_evd.json")
    c, _ = gpu_context(w)
    steps, delta, ok = c.converge(w.tol, 3000, n_check=10)
    assert ok, (steps, delta)
    e, _ = c.energy(ci.site_energy_operator(w))
    c.close()
    assert abs(e - gold["e_site"]) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16", 5e-2)])
def test_mixed_precision_energy_error(prec, tol):
    w = ci.WORKLOADS["c2"]
    gold = _gold("c2_qr.json")
    c, _ = gpu_context(w, prec=prec)
    c.step(gold["steps"])
    e, _ = c.energy(ci.site_energy_operator(w))
    c.close()
    print(f"{prec}: |dE| = {abs(e - gold['e_site']):.3e}")
    assert abs(e - gold["e_site"]) < tol


def test_converge_reports_steps_and_delta():
    w = ci.WORKLOADS["c1"]
    c, _ = gpu_context(w)
    steps, delta, ok = c.converge(1e-6, 200, n_check=5)
    assert ok and delta < 1e-6 and steps % 5 == 0 and steps <= 200
    x, st, pr = c.query()
    assert st == steps and x == w.chi and pr == w.chi * w.D2
    steps2, delta2, ok2 = c.converge(1e-30, 3, n_check=1)
    assert not ok2 and steps2 == 3
    c.close()


def test_precision_ladder_reaches_fp64_energy():
    """BF16 -> FP32 -> FP64 ladder on the D=4, chi=64 Kitaev workload: the
    converged energy is the FP64 one."""
    w = ci.WORKLOADS["c2"]
    gold = _gold("c2_qr.json")
    c, _ = gpu_context(w, prec="ladder")
    steps, delta, ok = c.converge(w.tol, 4000, n_check=10)
    e, _ = c.energy(ci.site_energy_operator(w))
    c.close()
    print(f"ladder: {steps} steps, |dE| = {abs(e - gold['e_site']):.3e}")
    assert ok and delta < w.tol
    assert abs(e - gold["e_site"]) < 1e-10


def test_update_tensor_continues_from_the_environment():
    """ctm_update_tensor keeps C, T, P_prev: the continued run equals a fresh
    context with the new tensor started from the same environment; a
    tensor that is not C3v-symmetric is rejected and changes nothing."""
    w = ci.Workload("u", 2, 3, 20, 301, 302)
    c, A = gpu_context(w)
    c.step(6)
    C0, T0, P0 = c.get_env()
    A2 = ctm.symmetrize(torch.tensor(ci.gaussian((2, 3, 3, 3), 303), device=DEV))
    bad = A2.clone()
    bad[0, 0, 1, 2] += 0.1
    with pytest.raises(ctm.CtmError):
        c.update_tensor(bad)
    C1, T1, P1 = c.get_env()
    assert torch.equal(C0, C1) and torch.equal(T0, T1) and torch.equal(P0, P1)
    c.update_tensor(A2)
    c.step(3)
    e1, _ = c.energy(ci.heisenberg_rotated())
    Cu, Tu, Pu = c.get_env()
    c.close()
    f = ctm.Context(A2, torch.tensor(ci.start_matrix(w), device=DEV), w.chi)
    f.set_env(C0, T0, P0)
    f.step(3)
    e2, _ = f.energy(ci.heisenberg_rotated())
    Cf, Tf, Pf = f.get_env()
    f.close()
    assert torch.equal(Cu, Cf) and torch.equal(Tu, Tf) and torch.equal(Pu, Pf)
    assert e1 == e2
