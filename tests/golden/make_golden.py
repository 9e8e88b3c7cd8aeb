"""Writes the stored oracle results under tests/golden/.

Calls only the CPU oracle (``oracle/``) and the seeded input generators.
Run from the repository root:

    python tests/golden/make_golden.py [c1 c2 c3 c4]

Each workload is iterated with the oracle's QR projector (and, for c2, also
with the eigendecomposition projector) until the corner-spectrum change falls
below the workload's tolerance or the step budget is used; the JSON records
the step count, the last change, the energies and the corner spectrum.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import ctm_inputs as ci  # noqa: E402
from oracle import ctm  # noqa: E402

MAX_STEPS = {"c1": 50, "c2": 3000, "c3": 4000, "c4": 3000}
CHECKPOINTS = (10, 20, 50, 100, 200, 400)
PROJECTORS = {"c1": ("qr",), "c2": ("qr", "evd"), "c3": ("qr",), "c4": ("qr",)}


def run(key: str, proj: str) -> dict:
    w = ci.WORKLOADS[key]
    A = ctm.prepare_site_tensor(ci.raw_site_tensor(w))
    G = ci.start_matrix(w)
    st = ctm.State(A, w.chi, G, proj=proj)
    ops = ci.bond_operators(w)
    h_site = ci.site_energy_operator(w)
    t0 = time.time()
    history = []
    at_steps = {}
    limit = w.steps if w.steps is not None else MAX_STEPS[key]
    for k in range(1, limit + 1):
        history.append(st.step())
        if k in CHECKPOINTS:
            at_steps[k] = st.energy(h_site)
        if w.steps is None and history[-1] < w.tol:
            break
    elapsed = time.time() - t0
    env = st.measurement_environment()
    rho = ctm.bond_density_matrix(st.C, st.T, st.A, env)
    e = {k: ctm.expectation(rho, v) for k, v in ops.items()}
    return {
        "workload": key,
        "projector": proj,
        "d": w.d, "D": w.D, "chi": w.chi,
        "seed_A": w.seed_A, "seed_A2": w.seed_A2, "eps": w.eps, "seed_G": w.seed_G,
        "model": w.model,
        "steps": st.steps,
        "last_delta": history[-1],
        "delta_history_tail": history[-10:],
        "tol": w.tol,
        "e_bond": e,
        "e_site": 0.5 * sum(e.values()),
        "e_site_at_step": at_steps,
        "rho": rho.tolist(),
        "spectrum": st.spectrum.tolist(),
        "oracle_seconds": elapsed,
        "gauge": st.gauge if proj == "qr" else None,
    }


def main(keys):
    for key in keys:
        for proj in PROJECTORS[key]:
            out = run(key, proj)
            path = os.path.join(ROOT, "tests", "golden", f"{key}_{proj}.json")
            with open(path, "w") as f:
                json.dump(out, f, indent=1)
            print(key, proj, out["steps"], out["last_delta"], out["e_site"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c4", "c3"])
