#!/usr/bin/env python3
"""Benchmark of QR-based C3v CTMRG on one MI355X.

Workload: honeycomb iPEPS, d=2, D=6, chi=144 (enlarged corner 5184 x 5184),
seeded C3v-symmetrized Gaussian site tensor A = sym(G0 + 1e-2 G1) (seeds
1003, 1004), rotated spin-1/2 Heisenberg bond energy.  A step is one CTMRG
iteration: enlarged corner, reduced corner, FP64 QR projector with its basis
tied to the previous one, corner and edge renormalization.

The headline `value` is the mixed-precision rate (FP32 matrix-core
contractions with FP32 accumulation; QR, basis, normalization and energy in
FP64); FP64 and BF16 rates are reported beside it, with each mode's energy
and corner-spectrum error against the CPU oracle's stored run of the same
number of steps.  Timed steps are bracketed by stream synchronization and
run with the inputs resident in HBM.  The roofline figure is for the
(chi D^2) x chi x (chi D^2) matrix-core kernels, timed with HIP events on the
library's stream.  The CPU baseline times the oracle itself on the host for
a bounded sample of full-size steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_rate(ctm, torch, A, G, chi, prec, warmup, steps, n_check=10):
    """Steps/s of `steps` timed steps after `warmup` untimed ones; also the
    rate with the corner-spectrum check every n_check steps, and the stage
    profile of 10 further steps."""
    with ctm.Context(A, G, chi, prec=prec) as c:
        c.step(max(warmup, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(n_check, steps - done)
            c.step(k, delta=True)
            done += k
        torch.cuda.synchronize()
        dt_check = time.perf_counter() - t1
        c.profile(True)
        c.step(10)
        stages, flops = c.profile_read()
        c.profile(False)
    return steps / dt, steps / dt_check, stages, flops


def gpu_energy(ctm, torch, A, G, chi, prec, nsteps, h):
    with ctm.Context(A, G, chi, prec=prec) as c:
        c.step(nsteps)
        e, _ = c.energy(h)
        s = c.spectrum()
    return e, s


def cpu_baseline(w, sample_steps):
    """The oracle on the host: `sample_steps` full-size steps after the two
    growth steps, reported as steps/s."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import ctm_inputs as ci
    from oracle import ctm as oracle

    A = oracle.prepare_site_tensor(ci.raw_site_tensor(w))
    st = oracle.State(A, w.chi, ci.start_matrix(w))
    st.run(steps=2)
    t0 = time.perf_counter()
    st.run(steps=sample_steps)
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"value": sample_steps / dt, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample_steps} full-size QR-CTMRG steps (n = {w.n}) of the same workload, "
                      f"after the 2 growth steps; NumPy float64 with {threads} BLAS threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="fp32,fp64,bf16")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the CTMRG iteration is a sequential fixed-point map and "
              f"this build runs it on a single MI355X (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import ctm_inputs as ci
    from paper_2509_05090_amd import ctm

    w = ci.WORKLOADS["c3"]
    dev = torch.device("cuda:0")
    raw = torch.tensor(ci.raw_site_tensor(w), device=dev)
    A = ctm.symmetrize(raw)
    G = torch.tensor(ci.start_matrix(w), device=dev)
    h = ci.site_energy_operator(w)
    gold_path = os.path.join(ROOT, "tests", "golden", "c3_qr.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None

    modes = args.modes.split(",")
    res = {}
    for prec in modes:
        log(f"[bench] {prec}: warmup {args.warmup}, timing {args.steps} steps")
        rate, rate_check, stages, flops = gpu_rate(ctm, torch, A, G, w.chi, prec, args.warmup,
                                                   args.steps)
        r = {"iters_per_s": rate, "iters_per_s_with_check10": rate_check,
             "stage_ms_per_step": {k: v[0] / 10 for k, v in stages.items()}}
        big_ms, big_n = stages["big_gemm"]
        r["big_gemm"] = {"launches": big_n, "avg_ms": big_ms / max(big_n, 1),
                         "flops_per_launch": flops / max(big_n, 1),
                         "tflops": flops / (big_ms * 1e-3) / 1e12 if big_ms > 0 else None}
        if gold is not None:
            e, s = gpu_energy(ctm, torch, A, G, w.chi, prec, gold["steps"], h)
            r["e_site"] = e
            r["e_err_vs_oracle"] = abs(e - gold["e_site"])
            so = np.array(gold["spectrum"])
            m = min(len(s), len(so))
            r["spectrum_err_vs_oracle"] = float(np.abs(s[:m] - so[:m]).max())
            r["oracle_steps"] = gold["steps"]
        res[prec] = r
        log(f"[bench] {prec}: {json.dumps(r)}")

    head = "fp32" if "fp32" in res else modes[0]
    hr = res[head]
    bg = hr["big_gemm"]
    achieved = bg["tflops"]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[head],
                "unit": "TFLOP/s", "frac": (achieved / PEAK_TFLOPS[head]) if achieved else None,
                "traffic": None,
                "kernel": f"gemm_kernel<{head}> on the {w.n} x {w.chi} x {w.n} products "
                          f"(W, M, Gm, V2 and the transposed T' product)",
                "avg_launch_ms": bg["avg_ms"], "flops_per_launch": bg["flops_per_launch"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_sample)
    out = {
        "metric": "CTMRG iters/sec at D=6,chi=144 (mixed vs FP64) + energy err vs FP64 oracle",
        "value": hr["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / hr["iters_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else ("f64" if head == "fp64" else "bf16"),
        "data": "synthetic",
        "config": {"workload": "honeycomb iPEPS QR-CTMRG, d=2 D=6 chi=144, "
                               "A=sym(G0+1e-2 G1) seeds 1003/1004, start matrix seed 1010, "
                               "rotated Heisenberg",
                   "d": w.d, "D": w.D, "chi": w.chi, "n": w.n,
                   "precision": "contractions FP32 matrix cores (FP32 accumulate); "
                                "QR, basis, normalization, energy FP64"},
        "modes": res,
        "speedup_mixed_vs_fp64": (res["fp32"]["iters_per_s"] / res["fp64"]["iters_per_s"])
        if "fp32" in res and "fp64" in res else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
