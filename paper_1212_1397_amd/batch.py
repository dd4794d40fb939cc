"""The many-solve workload (batch_workload: 96 problems of uneven size,
wavenumber and face pattern) solved as a batch and one by one.  Every step
runs in the HIP library; this module only orders the calls.

    python -m paper_1212_1397_amd.batch [--count 96] [--streams 4] [--no-graphs] [--lanes 2]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import helmholtz6 as h6
from .workloads import batch_workload


def run(count: int = 96, streams: int = 4, graphs=True, tune: bool = True, seed: int = 4,
        log=None, lanes: int = 2):
    """Seconds for the sequential plain solves, for the batched solves on
    concurrent streams and for the queued form (one captured graph, a
    device-side queue per grid shape, `lanes` lanes per shape; the lanes and
    the graph are built once, untimed, and the build time is reported), all
    mixed FGMRES(30) to 1e-8, with iteration counts and agreement."""
    insts = batch_workload(count, seed)
    plans, Fs = [], []
    for inst in insts:
        p = h6.Plan(inst.n, inst.h, inst.k, inst.bc, precision="mixed")
        plans.append(p)
        Fs.append(p.rhs_gaussians(inst.centres, inst.amps, inst.sigma))
    kw = dict(method="fgmres", restart=30, tol=1e-8, maxit=600)
    # sequential, plain (no graphs, default tiles); one warm-up solve per distinct grid
    seen = set()
    for p, F in zip(plans, Fs):
        if p.dims not in seen:
            seen.add(p.dims)
            p.solve(F, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [p.solve(F, **kw) for p, F in zip(plans, Fs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # batched: autotuned tiles (one tuning per grid shape), graphs, concurrent streams
    if tune:
        import os
        cache = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "autotune.txt")
        for p in plans:
            p.autotune(cache)         # read back per grid shape and precision (timed once if absent)
    for p in plans:
        p.set_graphs(graphs)
    Us = [torch.zeros_like(F) for F in Fs]
    h6.solve_batch(plans, Fs, Us, nstreams=streams, **kw)    # warm-up: captures the step graphs
    for U in Us:
        U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = h6.solve_batch(plans, Fs, Us, nstreams=streams, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    worst = max(float(torch.linalg.norm(U - s[0]) / torch.linalg.norm(s[0])) for U, s in zip(Us, seq))
    its = [i["iters"] for i in infos]
    # queued form: one graph, device-side queue per grid shape (from U = 0);
    # the lanes and the graph are built once (like the step graphs above)
    Uq = [torch.zeros_like(F) for F in Fs]
    t0 = time.perf_counter()
    queue = h6.Queue(plans, restart=30, lanes=lanes)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    queue.solve(Fs, Uq, tol=1e-8, maxit=600)                                             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qinfos = queue.solve(Fs, Uq, tol=1e-8, maxit=600)
    torch.cuda.synchronize()
    t_queue = time.perf_counter() - t0
    queue.close()
    qworst = max(float(torch.linalg.norm(U - s[0]) / torch.linalg.norm(s[0])) for U, s in zip(Uq, seq))
    qits = [i["iters"] for i in qinfos]
    res = {"count": count, "streams": streams, "graphs": graphs, "autotuned": tune,
           "unknowns": int(sum(p.dims[0] * p.dims[1] * p.dims[2] for p in plans)),
           "sequential_s": round(t_seq, 4), "batched_s": round(t_batch, 4),
           "speedup": round(t_seq / t_batch, 3), "solves_per_s": round(count / t_batch, 2),
           "iters_min": min(its), "iters_max": max(its), "iters_total": sum(its),
           "all_converged": all(i["status"] == "ok" for i in infos),
           "max_rel_diff_vs_sequential": worst,
           "queued": {"lanes_per_shape": lanes, "s": round(t_queue, 4), "build_s": round(t_build, 4),
                      "speedup_vs_sequential": round(t_seq / t_queue, 3), "solves_per_s": round(count / t_queue, 2),
                      "iters_total": sum(qits), "all_converged": all(i["status"] == "ok" for i in qinfos),
                      "max_rel_diff_vs_sequential": qworst}}
    for p in plans:
        p.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=96)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--cycle-graphs", action="store_true",
                    help="one graph per restart cycle (device Givens) instead of one per step")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--lanes", type=int, default=2, help="lanes per grid shape of the queued form")
    a = ap.parse_args(argv)
    graphs = False if a.no_graphs else ("cycle" if a.cycle_graphs else True)
    print(json.dumps(run(a.count, a.streams, graphs, not a.no_tune, lanes=a.lanes)), flush=True)


if __name__ == "__main__":
    main()
