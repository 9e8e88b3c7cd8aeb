"""Variational optimization of the site tensor, oracle side (test
infrastructure: imported only by tests/).

Sec. II.D: the energy of the converged environment is differentiated with
respect to the site tensor; Sec. III.B: the tensor is optimized with L-BFGS,
each energy evaluation taking a few warm-up CTMRG steps (no gradient) and k
tracked steps through which the gradient is taken.  The parameters are a
C3v-symmetric tensor `a`; the state is A = a / ||a|| (the energy does not
depend on the norm).  Each evaluation starts from the environment the
previous one reached after its warm-up steps, the first from the small
initial environment with `init_steps` steps.

The gradient with respect to `a` is the tracked-step gradient g = dE/dA
(already on the symmetric subspace and orthogonal to A, because E is
scale-invariant) divided by ||a||: dA/da = (I - A A^T) / ||a||.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ctm
from . import grad as ograd


class Evaluator:
    """E(a) and dE/da through k tracked steps, with the warm-started
    environment described in the module docstring."""

    def __init__(self, G, chi, h, k=2, warmup=10, init_steps=40):
        self.G, self.chi, self.h = G, chi, h
        self.k, self.warmup, self.init_steps = k, warmup, init_steps
        self.env = None
        self.calls = 0

    def state_for(self, A, env):
        st = ctm.State(A, self.chi, self.G)
        if env is None:
            st.run(steps=self.init_steps)
        else:
            st.C, st.T, st.P = env
            st.run(steps=self.warmup)
        return st

    def evaluate(self, a, env):
        """(E, dE/da, environment after the warm-up) from the given start."""
        nrm = np.linalg.norm(a)
        A = a / nrm
        st = self.state_for(A, env)
        e, g = ograd.gradient(A, st.C, st.T, st.P, self.chi, self.k, self.h)
        return e, g / nrm, (st.C, st.T, st.P)

    def __call__(self, a):
        e, g, self.env = self.evaluate(a, self.env)
        self.calls += 1
        return e, g


def lbfgs(a0, evaluator, iters, history=10):
    """L-BFGS (strong Wolfe line search) from a0 for `iters` iterations.
    Returns the final parameters and the energy of every evaluation."""
    p = torch.tensor(np.array(a0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.LBFGS([p], lr=1.0, max_iter=iters, history_size=history,
                            tolerance_grad=1e-12, tolerance_change=1e-14,
                            line_search_fn="strong_wolfe")
    energies = []

    def closure():
        opt.zero_grad()
        e, g = evaluator(p.detach().numpy())
        p.grad = torch.tensor(np.ascontiguousarray(g, dtype=np.float64))
        energies.append(e)
        return torch.tensor(e)

    opt.step(closure)
    return p.detach().numpy(), energies
