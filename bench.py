#!/usr/bin/env python3
"""Benchmark of QR-based C3v CTMRG on one MI355X.

Workload: honeycomb iPEPS, d=2, D=6, chi=144 (enlarged corner 5184 x 5184),
seeded C3v-symmetrized Gaussian site tensor A = sym(G0 + 1e-2 G1) (seeds
1003, 1004), start matrix seed 1010, rotated spin-1/2 Heisenberg energy.  A
step is one CTMRG iteration: enlarged corner, reduced corner, FP64 QR
projector with its basis tied to the previous one, corner and edge
renormalization.

The headline `value` is the mixed-precision rate (FP32 matrix-core
contractions with FP32 accumulation; QR, basis, normalization and energy in
FP64); FP64 and BF16 rates are reported beside it.  For each mode the run is
also converged to the workload tolerance and its energy and corner spectrum
are compared with the CPU oracle's converged run (tests/golden/c3_qr.json);
a ladder leg (BF16, then FP32, then FP64) reports the time to the FP64
tolerance against plain FP64.
Timed steps are bracketed by stream synchronization, inputs resident in
HBM.  The roofline figure is for the (chi D^2) x chi x (chi D^2) matrix-core
products, timed with HIP events on the library's stream; their HBM traffic
comes from the rocprofv3 counter summary in profiles/ when one was taken for
the current kernel.  A gradient leg times the fixed-point adjoint on the
D=4, chi=100 Kitaev-Heisenberg workload, and a large leg reports FP32 and
FP64 rates and the checkpointed gradient time at D=8, chi=256 (enlarged
corner 16384 x 16384), and a projector leg times one iteration with the QR
and with the eigendecomposition projector at D=5, chi=120, the shape of the
paper's comparison of the two, and an optimization leg runs L-BFGS on the
site tensor with the paper's 10 warm-up and 24 tracked steps per evaluation
at D=5, chi=120.  The CPU baseline times the oracle itself on the host for a
bounded sample of full-size steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
GEMM_KERNEL = {"fp64": "gemm_kernel<double", "fp32": "gemm_kernel<float", "bf16": "gemm_kernel<__bf16"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ctmrg_c3_big_gemm_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_stream(torch, proj):
    """Stream context for a run: the Cholesky projector overlaps work on
    CU-masked streams of its own, which needs the library's stream to be a
    stream other than the legacy default one (blocking streams synchronize
    with it); the Householder projector runs on the default stream."""
    import contextlib
    return torch.cuda.stream(torch.cuda.Stream()) if proj == "qr_chol" else contextlib.nullcontext()


def gpu_rate(ctm, torch, A, G, chi, prec, warmup, steps, n_check=10, proj="qr"):
    """Steps/s of `steps` timed steps after `warmup` untimed ones (from the
    truncated regime), also with the corner-spectrum check every n_check
    steps, and the stage profile of 10 further steps."""
    with run_stream(torch, proj), ctm.Context(A, G, chi, proj=proj, prec=prec) as c:
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


def gpu_converged(ctm, torch, A, G, chi, prec, tol, max_steps, h, residuals=None, proj="qr"):
    """Converge (spectrum check every 10 steps); energy, spectrum, steps, time.
    If `residuals` is a dict it receives the isometry residual max|P^T P - I|
    of the final projector, the fixed-point residual (the largest change of T
    and of the projector under one more step: the aligned basis makes them
    stationary element by element) and the largest change of C under that
    step.  The corner is not stationary element by element at these
    workloads: its spectrum comes in +-lambda pairs and C keeps turning
    within their two-dimensional eigenspaces (the oracle does the same),
    while its spectrum, T, P and the energy converge."""
    with run_stream(torch, proj), ctm.Context(A, G, chi, proj=proj, prec=prec) as c:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, delta, ok = c.converge(tol, max_steps, n_check=10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e, _ = c.energy(h)
        s = c.spectrum()
        if residuals is not None:
            C0, T0, P0 = c.get_env()
            eye = torch.eye(P0.shape[1], dtype=P0.dtype, device=P0.device)
            residuals["isometry"] = float((P0.T @ P0 - eye).abs().max().item())
            c.step(1)
            C1, T1, P1 = c.get_env()
            residuals["fixed_point"] = float(max((T1 - T0).abs().max().item(),
                                                 (P1 - P0).abs().max().item()))
            residuals["corner_change"] = float((C1 - C0).abs().max().item())
    return e, s, steps, delta, ok, dt


def gradient_leg(ctm, torch, ci, np, n_dirs):
    """Fixed-point gradient on the D=4, chi=100 KH workload: converge, time
    ctm_grad, and compare <g, v> with central differences (h = 1e-6) of
    converged energies along the first n_dirs seeded symmetric directions
    (each perturbed run starts from the converged environment)."""
    w = ci.WORKLOADS["c4"]
    h = ci.site_energy_operator(w)
    dev = torch.device("cuda:0")
    A = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(w), device=dev))
    G = torch.tensor(ci.start_matrix(w), device=dev)
    with ctm.Context(A, G, w.chi) as c:
        t0 = time.perf_counter()
        steps, delta, ok = c.converge(1e-14, 6000, n_check=20)
        torch.cuda.synchronize()
        t_conv = time.perf_counter() - t0
        c.grad(h, mode=0, tol=1e-12)  # allocates the adjoint workspace
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g, e, iters, gok = c.grad(h, mode=0, tol=1e-12)
        torch.cuda.synchronize()
        t_grad = time.perf_counter() - t1
        env = c.get_env()
    out = {"workload": "d=2 D=4 chi=100 Kitaev-Heisenberg phi=0.3pi, FP64",
           "converge_steps": steps, "converge_s": t_conv, "adjoint_steps": iters,
           "grad_ms": 1e3 * t_grad, "grad_converged": gok, "e_site": e,
           "grad_norm": float(torch.linalg.norm(g).item())}
    if n_dirs > 0:
        def energy_at(At):
            with ctm.Context(At, G, w.chi) as cc:
                cc.set_env(*env)
                cc.converge(1e-14, 6000, n_check=20)
                return cc.energy(h)[0]

        gn = g.cpu().numpy()
        errs = []
        for seed in ci.DIRECTION_SEEDS[:n_dirs]:
            vt = ctm.symmetrize(torch.tensor(ci.direction(w, seed), device=dev))
            vt = vt / torch.linalg.norm(vt)
            fd = (energy_at(A + 1e-6 * vt) - energy_at(A - 1e-6 * vt)) / 2e-6
            errs.append(abs(float(np.sum(gn * vt.cpu().numpy())) - fd))
        out.update({"fd_directions": n_dirs, "fd_step": 1e-6, "fd_max_abs_err": max(errs),
                    "fd_median_abs_err": float(np.median(errs))})
    return out


def cpu_baseline(w, sample_steps):
    """The oracle on the host: `sample_steps` full-size steps after the two
    growth steps, reported as steps/s."""
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


# Tag of the current big-product kernel variant; a stored traffic figure is
# used only if it was taken for this variant.
KERNEL_TAG = "nt-vec16"


def stored_traffic(prec):
    """HBM bytes per launch of the big products from the committed counter
    summary, if it covers this kernel: a line `traffic_bytes_per_launch
    <prec> <kernel tag> <bytes>` in profiles/ctmrg_c3_big_gemm_traffic.md."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        m = re.match(r"\s*traffic_bytes_per_launch\s+(\w+)\s+(\S+)\s+([0-9.eE+]+)", line)
        if m and m.group(1) == prec and m.group(2) == KERNEL_TAG:
            return float(m.group(3))
    return None


def copy_probe(torch):
    """A plain 512 MiB device-to-device copy: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def large_leg(ctm, torch, ci, steps, k_grad):
    """D=8, chi=256 (enlarged corner 16384 x 16384): rate of FP32 and FP64
    steps from the same start (after the two growth steps and one full-size
    step), and the time of the checkpointed gradient through k_grad tracked
    FP64 steps (the state is left unchanged by ctm_grad)."""
    w = ci.WORKLOADS["c5"]
    h = ci.site_energy_operator(w)
    dev = torch.device("cuda:0")
    A = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(w), device=dev))
    G = torch.tensor(ci.start_matrix(w), device=dev)
    out = {"workload": "d=2 D=8 chi=256 (n = 16384), A seed 1006, start matrix seed 1013, "
                       "rotated Heisenberg"}
    for prec in ("fp32", "fp64"):
        with ctm.Context(A, G, w.chi, prec=prec) as c:
            c.step(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            e, _ = c.energy(h)
            out[prec] = {"iters_per_s": steps / dt, "steps": steps, "e_site_after": e}
            if prec == "fp64" and k_grad > 0:
                c.grad(h, mode=1, tol=0.0)  # allocates the adjoint workspace
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                g, _, _, _ = c.grad(h, mode=k_grad, tol=0.0)
                torch.cuda.synchronize()
                out["gradient"] = {"tracked_steps": k_grad, "grad_ms": 1e3 * (time.perf_counter() - t1),
                                   "grad_norm": float(torch.linalg.norm(g).item()), "precision": "FP64"}
    out["speedup_fp32_vs_fp64"] = out["fp32"]["iters_per_s"] / out["fp64"]["iters_per_s"]
    return out


def projector_leg(ctm, torch, ci, steps):
    """Forward CTMRG iteration time with the QR projector and with the
    eigendecomposition projector, FP64, at D=5, chi=120 (n = 3000): the shape
    on which the paper compares the two (Sec. III.B, Fig. 5)."""
    w = ci.WORKLOADS["p5"]
    dev = torch.device("cuda:0")
    A = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(w), device=dev))
    G = torch.tensor(ci.start_matrix(w), device=dev)
    out = {"workload": "d=2 D=5 chi=120 (n = 3000), A seed 1007, start matrix seed 1014, FP64"}
    for proj in ("qr", "evd"):
        with ctm.Context(A, G, w.chi, proj=proj) as c:
            c.step(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        out[proj] = {"ms_per_iter": 1e3 * dt / steps, "steps": steps}
    out["evd_over_qr"] = out["evd"]["ms_per_iter"] / out["qr"]["ms_per_iter"]
    out["note"] = ("the eigendecomposition baseline is this library's unblocked Householder "
                   "tridiagonalization (two kernels per column, HBM-bound) with a host "
                   "tridiagonal eigensolver, not a tuned library eigensolver: the ratio is an "
                   "upper bound of the QR projector's gain")
    return out


def optimization_leg(ctm, torch, ci, iters):
    """L-BFGS on the site tensor at D=5, chi=120 with 10 warm-up and 24
    tracked CTMRG steps per evaluation (the paper's setting, Sec. III.B,
    Fig. 5): energies and time per evaluation."""
    from paper_2509_05090_amd import optimize
    w = ci.WORKLOADS["p5"]
    a0 = ctm.symmetrize(torch.tensor(ci.raw_site_tensor(w), device="cuda")).cpu().numpy()
    ev = optimize.Evaluator(torch.tensor(ci.start_matrix(w), device="cuda"), w.chi,
                            ci.site_energy_operator(w), k=24, warmup=10, init_steps=40)
    t0 = time.perf_counter()
    _, energies = optimize.lbfgs(a0, ev, iters=iters)
    dt = time.perf_counter() - t0
    ev.close()
    return {"workload": "d=2 D=5 chi=120 rotated Heisenberg, L-BFGS, 10 warm-up + 24 tracked "
                        "steps per evaluation (FP64)",
            "iterations": iters, "evaluations": ev.calls, "seconds": dt,
            "ms_per_evaluation": 1e3 * ev.seconds / max(ev.calls, 1),
            "e_site_first": energies[0], "e_site_last": energies[-1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--modes", default="fp32,fp64,bf16")
    ap.add_argument("--proj", default="qr_chol", choices=("qr", "qr_chol"),
                    help="QR projector: Q1 by Householder (qr) or by Cholesky QR (qr_chol)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP32 rate with the Householder projector")
    ap.add_argument("--no-large", action="store_true", help="skip the D=8, chi=256 leg")
    ap.add_argument("--no-projectors", action="store_true",
                    help="skip the QR vs eigendecomposition leg (D=5, chi=120)")
    ap.add_argument("--no-opt", action="store_true", help="skip the L-BFGS leg (D=5, chi=120)")
    ap.add_argument("--fd-dirs", type=int, default=20,
                    help="finite-difference directions of the gradient leg")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--large-grad-k", type=int, default=2)
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

    if args.copy_probe:
        copy_probe(torch)
    w = ci.WORKLOADS["c3"]
    dev = torch.device("cuda:0")
    raw = torch.tensor(ci.raw_site_tensor(w), device=dev)
    A = ctm.symmetrize(raw)
    G = torch.tensor(ci.start_matrix(w), device=dev)
    h = ci.site_energy_operator(w)
    gold_path = os.path.join(ROOT, "tests", "golden", "c3_qr.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    gold_ok = gold is not None and gold.get("last_delta", 1.0) < w.tol

    modes = args.modes.split(",")
    res = {}
    for prec in modes:
        log(f"[bench] {prec}: warmup {args.warmup}, timing {args.steps} steps")
        rate, rate_check, stages, flops = gpu_rate(ctm, torch, A, G, w.chi, prec, args.warmup,
                                                   args.steps, proj=args.proj)
        r = {"iters_per_s": rate, "iters_per_s_with_check10": rate_check,
             "stage_ms_per_step": {k: v[0] / 10 for k, v in stages.items()}}
        big_ms, big_n = stages["big_gemm"]
        r["big_gemm"] = {"launches": big_n, "avg_ms": big_ms / max(big_n, 1),
                         "flops_per_launch": flops / max(big_n, 1),
                         "tflops": flops / (big_ms * 1e-3) / 1e12 if big_ms > 0 else None}
        if not args.no_converge:
            tol = {"fp64": w.tol, "fp32": 1e-8, "bf16": 1e-4}[prec]
            resid = {}
            e, s, steps, delta, ok, dt = gpu_converged(ctm, torch, A, G, w.chi, prec, tol, 4000, h,
                                                       resid, proj=args.proj)
            r.update({"e_site": e, "converge_tol": tol, "converge_steps": steps,
                      "converge_delta": delta, "converged": ok, "converge_s": dt,
                      "isometry_residual": resid["isometry"],
                      "fixed_point_residual": resid["fixed_point"],
                      "corner_change_per_step": resid["corner_change"]})
            if gold_ok:
                so = np.array(gold["spectrum"])
                m = min(len(s), len(so))
                r["e_err_vs_oracle"] = abs(e - gold["e_site"])
                r["spectrum_err_vs_oracle"] = float(np.abs(s[:m] - so[:m]).max())
                r["oracle_steps"] = gold["steps"]
        res[prec] = r
        log(f"[bench] {prec}: {json.dumps(r)}")

    householder = None
    if args.proj == "qr_chol" and "fp32" in modes and not args.no_compare:
        log("[bench] fp32 with the Householder projector, for comparison")
        hrate, _, hstages, _ = gpu_rate(ctm, torch, A, G, w.chi, "fp32", args.warmup, args.steps,
                                        proj="qr")
        householder = {"fp32_iters_per_s": hrate,
                       "stage_ms_per_step": {k: v[0] / 10 for k, v in hstages.items()}}
        log(f"[bench] householder: {json.dumps(householder)}")

    ladder = None
    if not args.no_converge:
        log("[bench] ladder: BF16 -> FP32 -> FP64, converged to the FP64 tolerance")
        e, sl, steps, delta, ok, dt = gpu_converged(ctm, torch, A, G, w.chi, "ladder", w.tol, 6000, h,
                                                    proj=args.proj)
        ladder = {"converge_tol": w.tol, "converge_steps": steps, "converge_delta": delta,
                  "converged": ok, "converge_s": dt, "e_site": e}
        if gold_ok:
            so = np.array(gold["spectrum"])
            m = min(len(sl), len(so))
            ladder["e_err_vs_oracle"] = abs(e - gold["e_site"])
            ladder["spectrum_err_vs_oracle"] = float(np.abs(sl[:m] - so[:m]).max())
        if "fp64" in res and "converge_s" in res["fp64"]:
            ladder["time_to_solution_speedup_vs_fp64"] = res["fp64"]["converge_s"] / dt
        log(f"[bench] ladder: {json.dumps(ladder)}")

    grad = None
    if not args.no_grad:
        log("[bench] gradient leg (D=4, chi=100)")
        grad = gradient_leg(ctm, torch, ci, np, args.fd_dirs)
        log(f"[bench] gradient: {json.dumps(grad)}")

    large = None
    if not args.no_large:
        log("[bench] large leg (D=8, chi=256)")
        large = large_leg(ctm, torch, ci, args.large_steps, args.large_grad_k)
        log(f"[bench] large: {json.dumps(large)}")

    projectors = None
    if not args.no_projectors:
        log("[bench] projector leg: QR vs EVD at D=5, chi=120")
        projectors = projector_leg(ctm, torch, ci, 10)
        log(f"[bench] projectors: {json.dumps(projectors)}")

    opt = None
    if not args.no_opt:
        log("[bench] optimization leg: L-BFGS at D=5, chi=120")
        opt = optimization_leg(ctm, torch, ci, 4)
        log(f"[bench] optimization: {json.dumps(opt)}")

    head = "fp32" if "fp32" in res else modes[0]
    hr = res[head]
    bg = hr["big_gemm"]
    achieved = bg["tflops"]
    traffic = stored_traffic(head)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[head],
                "unit": "TFLOP/s", "frac": (achieved / PEAK_TFLOPS[head]) if achieved else None,
                "traffic": traffic,
                "kernel": f"{GEMM_KERNEL[head]}, false, true, ...> on the three {w.n} x {w.chi} x {w.n} "
                          f"products of a step (M = Ct P, Ct Q, V Q; the {w.chi}-wide operand "
                          f"stored transposed)",
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
                                "QR, basis, normalization, energy FP64",
                   "qr": "Q1 by Cholesky QR (3 passes), gs(X) by Householder"
                         if args.proj == "qr_chol" else "Householder"},
        "modes": res,
        "speedup_mixed_vs_fp64": (res["fp32"]["iters_per_s"] / res["fp64"]["iters_per_s"])
        if "fp32" in res and "fp64" in res else None,
        "householder_projector": householder,
        "ladder": ladder,
        "gradient": grad,
        "large": large,
        "projectors": projectors,
        "optimization": opt,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
