"""GPU variational optimization (paper_2509_05090_amd/optimize.py) against the
oracle driver (oracle/optimize.py): the same L-BFGS run from the same start,
every energy evaluation compared, and one evaluation's gradient with respect
to the unnormalized parameters element by element."""
import numpy as np
import pytest
import torch

import ctm_inputs as ci
from oracle import ctm as oracle
from oracle import optimize as oopt
from paper_2509_05090_amd import optimize as gopt

pytestmark = pytest.mark.gpu
H = 1.5 * ci.heisenberg_rotated()


def _setup(D, chi, seed):
    a = 2.5 * oracle.symmetrize(ci.gaussian((2, D, D, D), seed))
    G = ci.gaussian((chi * D * D, chi), seed + 1)
    return a, G


@pytest.mark.parametrize("D,chi,seed", [(2, 16, 51), (3, 20, 52)])
def test_evaluation_matches_oracle(D, chi, seed):
    a, G = _setup(D, chi, seed)
    ge = gopt.Evaluator(torch.tensor(G, device="cuda"), chi, H, k=2, warmup=10, init_steps=30)
    oe = oopt.Evaluator(G, chi, H, k=2, warmup=10, init_steps=30)
    for scale in (1.0, 1.001):  # second call: warm-started from the first
        eg, gg = ge(scale * a)
        eo, go = oe(scale * a)
        err = np.abs(gg - go).max() / np.abs(go).max()
        print(f"D={D} chi={chi}: |dE| {abs(eg - eo):.2e}, grad rel err {err:.2e}")
        assert abs(eg - eo) < 1e-12
        assert err < 1e-9


def test_lbfgs_trajectory_matches_oracle():
    """Four L-BFGS iterations at D=2, chi=16: the GPU and oracle drivers
    take the same line-search steps, so every evaluation agrees."""
    a, G = _setup(2, 16, 53)
    ge = gopt.Evaluator(torch.tensor(G, device="cuda"), 16, H, k=2, warmup=10, init_steps=30)
    oe = oopt.Evaluator(G, 16, H, k=2, warmup=10, init_steps=30)
    ag, eg = gopt.lbfgs(a, ge, iters=4)
    ao, eo = oopt.lbfgs(a, oe, iters=4)
    print("gpu", eg)
    print("oracle", eo)
    print(f"{ge.calls} GPU evaluations, {ge.seconds / ge.calls * 1e3:.1f} ms each")
    assert len(eg) == len(eo)
    assert np.abs(np.array(eg) - np.array(eo)).max() < 1e-9
    assert eg[-1] < eg[0] - 1e-3
    assert np.abs(ag - ao).max() < 1e-7 * np.abs(ao).max()
