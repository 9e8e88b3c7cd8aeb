"""Pins of the oracle's variational optimization driver (oracle/optimize.py):
the chain rule through the normalization A = a / ||a|| against central
differences of the driver's own energy (starting environment held fixed,
no warm-up steps), and descent of the L-BFGS iteration."""
import numpy as np

import ctm_inputs as ci
from oracle import ctm
from oracle import optimize as oopt

H = 1.5 * ci.heisenberg_rotated()


def _setup(D=2, chi=8, seed=31):
    a = 3.7 * ctm.symmetrize(ci.gaussian((2, D, D, D), seed))
    G = ci.gaussian((chi * D * D, chi), seed + 1)
    return a, G, chi


def test_gradient_wrt_unnormalized_parameters_matches_differences():
    a, G, chi = _setup()
    ev = oopt.Evaluator(G, chi, H, k=2, warmup=0, init_steps=30)
    _, _, env = ev.evaluate(a, None)
    e0, g, _ = ev.evaluate(a, env)
    assert abs(np.sum(g * a)) < 1e-12 * np.abs(g).max() * np.linalg.norm(a)  # scale invariance
    h = 1e-6
    for seed in (41, 42, 43):
        v = ctm.symmetrize(ci.gaussian(a.shape, seed))
        fd = (ev.evaluate(a + h * v, env)[0] - ev.evaluate(a - h * v, env)[0]) / (2 * h)
        assert abs(np.sum(g * v) - fd) < 1e-8 * max(1.0, abs(fd)), (np.sum(g * v), fd)


def test_lbfgs_descends():
    a, G, chi = _setup()
    ev = oopt.Evaluator(G, chi, H, k=2, warmup=10, init_steps=30)
    _, energies = oopt.lbfgs(a, ev, iters=4)
    print("energies", energies)
    assert len(energies) >= 4
    assert energies[-1] < energies[0] - 1e-3
