"""Benchmark: seconds to a 1e-8 relative residual on the 256^3 mixed-face
Helmholtz problem (sixth-order compact scheme, 7-point FFT preconditioner),
plain FP64 GMRES(30) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dns-256]

One step is one complete solve (all hot-path stages: right-hand side resident
in HBM, GMRES Arnoldi steps with preconditioner and operator applications,
modified Gram-Schmidt, cycle updates and true-residual checks).  Warm-up
solves are untimed; then K solves are timed between two device
synchronisations.  Rank 0 prints one JSON line with:
  value / ms_per_step  - seconds / milliseconds per solve (lower is better),
  roofline             - the kernel with the largest share of the solve time,
                         its algorithmic HBM bytes per launch over its average
                         launch duration (HIP events on the solve's stream),
  cpu_baseline         - the FP64 CPU oracle on a bounded sample of the same
                         solve, scaled to a whole solve.
Secondary figures (SKS, per-kernel bandwidths) ride along in "extra".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(plan, cls: str, n_unknowns: int, elem: int = 16) -> float:
    """Bytes one launch of a kernel class must move at minimum (per unknown x N).

    stencil: read x, write y (2 vectors); stencil_resid: read x and F, write r
    (3); each transform pass and the z solve: read and write one vector (2).
    """
    per = {"stencil": 2, "stencil_resid": 3, "xform_x": 2, "xform_y": 2, "tridiag_z": 2}[cls]
    return float(per * elem * n_unknowns)


def run_cpu_baseline(w, gpu_iters: int):
    """Oracle GMRES on the same problem, stopped after two Arnoldi steps, scaled
    to the GPU's iteration count (the oracle's per-step cost is uniform)."""
    import numpy as np

    import oracle
    from oracle.functions import gaussian_sources
    from paper_1212_1397_amd.workloads import gaussian_sources as wl_sources

    prob = oracle.Problem.cube(w.n, w.k, w.bc)
    centres, amps, sigma = wl_sources(w)
    F = oracle.rhs(prob, gaussian_sources(centres, amps, sigma))
    t0 = time.perf_counter()
    _, info = oracle.solve(prob, F, "gmres", restart=w.restart, tol=w.tol, maxit=2)
    dt = time.perf_counter() - t0
    per_iter = dt / max(info.iters, 1)
    return {"value": per_iter * gpu_iters, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle GMRES({w.restart}) on the full {w.name} grid stopped after "
                      f"{info.iters} Arnoldi steps (incl. initial and cycle-end residuals): "
                      f"{dt:.1f} s, scaled to {gpu_iters} steps; numpy/scipy single-threaded",
            "sample_seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dns-256")
    ap.add_argument("--method", default="gmres", choices=["gmres", "sks", "fgmres"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1212_1397_amd import helmholtz6 as h6
    from paper_1212_1397_amd.workloads import WORKLOADS, gaussian_sources

    w = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    plan = h6.Plan(w.n, w.h, w.k, w.bc)
    N = plan.dims[0] * plan.dims[1] * plan.dims[2]
    centres, amps, sigma = gaussian_sources(w)
    F = plan.rhs_gaussians(centres, amps, sigma)
    U = torch.zeros_like(F)
    print(f"# workload {w.name}: dims {plan.dims}, N = {N}, k = {w.k}, bc = {w.bc}", file=sys.stderr,
          flush=True)

    def one_solve(method):
        U.zero_()
        _, info = plan.solve(F, U, method=method, restart=w.restart, tol=w.tol, maxit=500)
        if info["status"] != "ok":
            raise RuntimeError(f"solve did not converge: {info}")
        return info

    for _ in range(args.warmup):
        info = one_solve(args.method)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = one_solve(args.method)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(f"# timed {args.steps} solves: {dt * 1e3:.2f} ms/solve, {info['iters']} iterations, "
          f"rel resid {info['rel_resid']:.3e}", file=sys.stderr, flush=True)

    # per-kernel durations from HIP events on the solve's stream (one extra solve)
    plan.profile(True)
    for c in h6.KERNEL_CLASSES:
        plan.kernel_time(c, reset=True)
    one_solve(args.method)
    torch.cuda.synchronize()
    ktimes = {c: plan.kernel_time(c) for c in h6.KERNEL_CLASSES}
    plan.profile(False)
    total_ms = sum(ms for ms, _ in ktimes.values())
    kernels = {}
    for c, (ms, n) in ktimes.items():
        if n == 0:
            continue
        rec = {"ms_total": ms, "launches": n, "avg_us": 1e3 * ms / n, "share": ms / total_ms}
        if c in ("stencil", "stencil_resid", "xform_x", "xform_y", "tridiag_z"):
            b = algorithmic_bytes(plan, c, N)
            rec["alg_bytes_per_launch"] = b
            rec["gbs"] = b / (1e-3 * ms / n) / 1e9
            rec["frac_hbm"] = rec["gbs"] / HBM_PEAK_GBS
        kernels[c] = rec
    bw = {c: r for c, r in kernels.items() if "gbs" in r}
    dom = max(bw, key=lambda c: bw[c]["ms_total"])
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(bw[dom]["gbs"], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(bw[dom]["frac_hbm"], 4),
                "traffic": None}

    extra = {"kernels": kernels}
    if not args.no_extra and args.method == "gmres":
        t1 = time.perf_counter()
        si = one_solve("sks")
        torch.cuda.synchronize()
        extra["sks"] = {"s": time.perf_counter() - t1, "iters": si["iters"], "rel_resid": si["rel_resid"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(w, info["iters"])

    out = {
        "metric": "s to 1e-8 resid @256^3: mixed/learned vs plain FP64 GPU; stencil+precond HBM GB/s",
        "value": round(dt, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid_unknowns": list(plan.dims), "interior_nodes": w.n,
                   "k": [w.k.real, w.k.imag], "faces": w.bc, "sources": w.nsrc,
                   "method": f"{args.method}({w.restart})" if args.method != "sks" else "sks",
                   "precision": "fp64", "tol": w.tol, "iterations": info["iters"],
                   "rel_resid": info["rel_resid"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
