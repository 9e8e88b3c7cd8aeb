"""Variational optimization of the site tensor on the GPU.

Sec. II.D: the energy of the converged environment is differentiated with
respect to the site tensor; Sec. III.B: the tensor is optimized with L-BFGS,
each energy evaluation taking a few warm-up CTMRG steps (no gradient) and k
tracked steps through which the gradient is taken (ctm_grad mode k).  The
parameters are a C3v-symmetric tensor `a`; the state is A = a / ||a||.
Each evaluation starts from the environment the previous one reached after
its warm-up steps: one context serves the whole run, its site tensor
replaced per evaluation (ctm_update_tensor); the first evaluation starts
from the small initial environment with `init_steps` steps.

Every CTMRG step, energy and gradient runs in libctm; the L-BFGS update
itself acts on the d D^3 parameters on the host.  dE/da = (dE/dA) / ||a||
because ctm_grad's result is on the symmetric subspace and orthogonal to A
(the energy does not depend on the norm of A).
"""
from __future__ import annotations

import time

import numpy as np

from . import ctm


class Evaluator:
    """E(a) and dE/da through k tracked steps on the GPU."""

    def __init__(self, G, chi, h, k=2, warmup=10, init_steps=40):
        import torch
        self.torch = torch
        self.G = G if isinstance(G, torch.Tensor) else torch.tensor(G, device="cuda")
        self.chi, self.h = chi, np.asarray(h, dtype=np.float64)
        self.k, self.warmup, self.init_steps = k, warmup, init_steps
        self.ctx = None
        self.calls = 0
        self.seconds = 0.0

    def __call__(self, a):
        torch = self.torch
        t0 = time.perf_counter()
        nrm = float(np.linalg.norm(a))
        A = torch.tensor(np.asarray(a, dtype=np.float64) / nrm, device="cuda")
        if self.ctx is None:
            self.ctx = ctm.Context(A, self.G, self.chi)
            self.ctx.step(self.init_steps)
        else:
            self.ctx.update_tensor(A)
            self.ctx.step(self.warmup)
        g, e, _, _ = self.ctx.grad(self.h, mode=self.k)  # leaves the environment as it was
        gh = g.cpu().numpy() / nrm
        self.calls += 1
        self.seconds += time.perf_counter() - t0
        return e, gh

    def close(self):
        if self.ctx is not None:
            self.ctx.close()
            self.ctx = None


def lbfgs(a0, evaluator, iters, history=10):
    """L-BFGS (strong Wolfe line search) from a0 for `iters` iterations.
    Returns the final parameters and the energy of every evaluation."""
    import torch
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
