"""Training data, training and evaluation of the learned correction
(include/h6net.h).  Every step runs in the HIP library; this module only
orders the calls.

Training pairs come from plain solves (the stationary SKS iteration of
Algorithm 1 on the complex64-preconditioned plan): for a problem A U = F with
reference solution U* (flexible GMRES to 1e-11) and SKS iterates U_j, the
residual r_j = F - A U_j and error e_j = U* - U_j satisfy A e_j = r_j; the
network is trained to output t_j = e_j - A_p^{-1} r_j, what the plain
preconditioner misses.  Two losses: "plain", |c(r) - t|^2 / |t|^2, and
"operator", |A (c(r) - t)|^2 / |A t|^2.  Since A t = r - A A_p^{-1} r, the
operator loss is the squared ratio of the residual of the corrected
preconditioner to that of the plain one, the quantity by which the flexible
solver accepts or rejects a correction.

    python -m paper_1212_1397_amd.learned train --out weights.npz [--n 128] [--problems 16]
                                              [--iters 8] [--steps 1500] [--seed 4]
                                              [--loss plain|operator] [--init weights.npz]
                                              [--stream --steps-per-problem 8 --buffer 8]
    python -m paper_1212_1397_amd.learned eval  --weights weights.npz [--workload dns-256]
    python -m paper_1212_1397_amd.learned speed [--workload dns-256]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import helmholtz6 as h6
from .workloads import WORKLOADS, gaussian_sources, init_net_params, random_sources

BC = "DDNNSS"


def problem(n: int, seed: int):
    """A seeded training problem: k = kr (1 + 0.01 i), kr ~ U[20, 80], 1-8 Gaussian sources."""
    rng = np.random.default_rng(seed)
    kr = float(rng.uniform(20.0, 80.0))
    nsrc = int(rng.integers(1, 9))
    h = 1.0 / (n + 1)
    return kr * (1 + 0.01j), random_sources(nsrc, seed + 1000, h), h


def problem_pairs(n: int, seed: int, iters: int):
    """One seeded problem: its plan, k, h, the reference solve's info and the
    pairs [(r_j, t_j)] of the SKS iterates U_0 = 0, U_1, ..., U_{iters-1}
    (formed by h6net_training_pair)."""
    k, (centres, amps, sigma), h = problem(n, seed)
    plan = h6.Plan(n, h, k, BC, precision="mixed")
    F = plan.rhs_gaussians(centres, amps, sigma)
    Us, info = plan.solve(F, method="fgmres", restart=30, tol=1e-11, maxit=400)
    U = torch.zeros_like(F)
    pairs = []
    for j in range(iters):
        if j > 0:       # U_j = U_{j-1} + A_p^{-1} (F - A U_{j-1}): one SKS step from U_{j-1}
            plan.solve(F, U, method="sks", tol=0.0, maxit=1, zero_guess=False)
        pairs.append(plan.training_pair(F, Us, U))
    return plan, k, h, info, pairs


def make_pairs(n: int, nproblems: int, iters: int, seed: int, log=print, keep_plans: bool = False):
    """[(r, t, kh, plan)] on the GPU from plain solves of `nproblems` seeded
    problems; plan is the problem's (open) plan if keep_plans, else None."""
    out = []
    for p in range(nproblems):
        plan, k, h, info, pairs = problem_pairs(n, seed + p, iters)
        kh = k.real * h
        out += [(r, t, kh, plan if keep_plans else None) for r, t in pairs]
        log(f"problem {p}: k = {k:.2f}, reference {info['iters']} FGMRES steps "
            f"(rel resid {info['rel_resid']:.1e}), {iters} pairs")
        if not keep_plans:
            plan.close()
    return out


def train_stream(net: h6.Net, n: int, problems: int, iters: int, seed: int, steps_per_problem: int,
                 buffer: int = 8, lr0: float = 1e-3, loss: str = "operator", log=print):
    """Training on a stream of `problems` seeded problems (problems x iters
    pairs in all): each new problem's pairs join a buffer of the last
    `buffer` problems, and `steps_per_problem` Adam steps follow, each on a
    pair drawn at random from the buffer (cosine learning-rate decay over the
    whole run).  Returns the loss history and the seconds spent."""
    from collections import deque
    rng = np.random.default_rng(seed)
    buf = deque()
    total = problems * steps_per_problem
    hist, step = [], 0
    t0 = time.perf_counter()
    for p in range(problems):
        plan, k, h, info, pairs = problem_pairs(n, seed + p, iters)
        buf.append((plan, k.real * h, pairs))
        if len(buf) > buffer:
            buf.popleft()[0].close()
        for _ in range(steps_per_problem):
            lr = lr0 * 0.5 * (1 + np.cos(np.pi * step / total)) + 1e-5
            pl, kh, prs = buf[int(rng.integers(len(buf)))]
            r, t = prs[int(rng.integers(len(prs)))]
            want = step % 250 == 0 or step == total - 1
            if loss == "operator":
                L = net.train_step_op(pl, r, t, lr, want_loss=want)
            else:
                L = net.train_step(r, kh, t, lr, want_loss=want)
            if want:
                hist.append((step, L))
                log(f"step {step} (problem {p}, {(p + 1) * iters} pairs): loss {L:.4f} lr {lr:.2e} "
                    f"({time.perf_counter() - t0:.1f} s)")
            step += 1
    for pl, _, _ in buf:
        pl.close()
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def train(net: h6.Net, pairs, steps: int, lr0: float = 1e-3, seed: int = 0, log=print, loss: str = "plain"):
    """Adam over randomly drawn pairs with a cosine learning-rate decay; returns
    the loss history.  loss = "operator" needs pairs made with keep_plans."""
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        lr = lr0 * 0.5 * (1 + np.cos(np.pi * s / steps)) + 1e-5
        r, t, kh, plan = pairs[int(rng.integers(len(pairs)))]
        want = s % 25 == 0 or s == steps - 1
        if loss == "operator":
            L = net.train_step_op(plan, r, t, lr, want_loss=want)
        else:
            L = net.train_step(r, kh, t, lr, want_loss=want)
        if want:
            hist.append((s, L))
            log(f"step {s}: loss {L:.4f} lr {lr:.2e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def pair_losses(net: h6.Net, pairs, operator: bool = False):
    """Per pair (|c(r) - t|, |t|): the error of the corrected preconditioner
    A_p^{-1} r + c(r) against e, and that of the plain one (t = e - A_p^{-1} r);
    with operator, (|A (c - t)|, |A t|): the residuals of the two
    preconditioners (pairs made with keep_plans)."""
    out = []
    for r, t, kh, plan in pairs:
        c = net.forward(r, kh)
        if operator:
            out.append((float(torch.linalg.norm(plan.apply_A(c - t))), float(torch.linalg.norm(plan.apply_A(t)))))
        else:
            out.append((float(torch.linalg.norm(c - t)), float(torch.linalg.norm(t))))
    return out


def solve_compare(w, params, log=print):
    """Mixed FGMRES(30) on workload `w` with and without the correction."""
    plan = h6.Plan(w.n, w.h, w.k, w.bc, precision="mixed")
    F = plan.rhs_gaussians(*gaussian_sources(w))

    def timed(attach):
        plan.attach_net(attach)
        U = torch.zeros_like(F)
        plan.solve(F, U, method="fgmres", restart=w.restart, tol=w.tol, maxit=500)    # warm-up
        torch.cuda.synchronize()
        U.zero_()
        t0 = time.perf_counter()
        U, info = plan.solve(F, U, method="fgmres", restart=w.restart, tol=w.tol, maxit=500)
        torch.cuda.synchronize()
        return U, info, time.perf_counter() - t0

    U0, i0, t0 = timed(None)
    net = h6.Net(plan.dims)
    net.set_params(params)
    U1, i1, t1 = timed(net)
    steps = plan.learned_steps()
    plan.attach_net(None)
    diff = float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0))
    res = {"workload": w.name, "plain": {"iters": i0["iters"], "s": round(t0, 6), "rel_resid": i0["rel_resid"]},
           "learned": {"iters": i1["iters"], "s": round(t1, 6), "rel_resid": i1["rel_resid"],
                       "steps_with_correction": steps},
           "solution_rel_diff": diff}
    log(json.dumps(res))
    return res


def net_flops(dims) -> float:
    """Multiply-add flops (2 per MAC) of one forward pass on grid `dims`
    (input layer counted with its 3 real channels)."""
    g1 = list(dims)
    g2 = [(x + 1) // 2 for x in g1]
    g3 = [(x + 1) // 2 for x in g2]
    P = [float(np.prod(g)) for g in (g1, g2, g3)]
    level = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "b3a": 2, "b3b": 2, "d2a": 1, "d2b": 1,
             "d1a": 0, "d1b": 0, "out": 0}
    return sum(2.0 * 27 * ci * co * P[level[name]] for name, ci, co in h6.NET_LAYERS)


def speed(dims, reps: int = 5, train: bool = False):
    """Average seconds of a forward pass (or training step) on `dims` and the
    achieved TFLOP/s (a training step counted as three forward passes)."""
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(init_net_params(h6.NET_LAYERS, 1)))
    shape = (dims[2], dims[1], dims[0])
    g = torch.Generator(device="cuda").manual_seed(0)
    r = torch.randn(shape, dtype=torch.complex128, device="cuda", generator=g)
    t = torch.randn(shape, dtype=torch.complex128, device="cuda", generator=g)
    run = (lambda: net.train_step(r, 0.3, t, 1e-5, want_loss=False)) if train else (lambda: net.forward(r, 0.3))
    run()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        run()
    b.record()
    b.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    fl = net_flops(dims) * (3.0 if train else 1.0)
    return sec, fl / sec / 1e12


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--n", type=int, default=128)
    t.add_argument("--problems", type=int, default=16)
    t.add_argument("--iters", type=int, default=8)
    t.add_argument("--steps", type=int, default=1500)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=4)
    t.add_argument("--holdout", type=int, default=2)
    t.add_argument("--loss", choices=("plain", "operator"), default="plain")
    t.add_argument("--init", default=None, help="start from these weights (.npz) instead of a seeded init")
    t.add_argument("--stream", action="store_true",
                   help="generate the problems' pairs while training (a buffer of recent problems) "
                        "instead of holding every pair")
    t.add_argument("--steps-per-problem", type=int, default=8)
    t.add_argument("--buffer", type=int, default=8)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--workload", default="dns-256")
    sp = sub.add_parser("speed")
    sp.add_argument("--workload", default="dns-256")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.cmd == "train":
        op = args.loss == "operator"
        held = make_pairs(args.n, args.holdout, args.iters, args.seed + 10_000, log, keep_plans=True)
        dims = tuple(held[0][0].shape[::-1])
        net = h6.Net(dims)
        if args.init:
            net.set_params(np.load(args.init)["params"])
        else:
            net.set_params(h6.pack_net_params(init_net_params(h6.NET_LAYERS, args.seed)))
        before = [a / b for a, b in pair_losses(net, held, operator=True)]
        if args.stream:
            hist, secs = train_stream(net, args.n, args.problems, args.iters, args.seed, args.steps_per_problem,
                                      args.buffer, args.lr, args.loss, log)
            steps = args.problems * args.steps_per_problem
        else:
            pairs = make_pairs(args.n, args.problems, args.iters, args.seed, log, keep_plans=op)
            hist, secs = train(net, pairs, args.steps, args.lr, args.seed, log, loss=args.loss)
            steps = args.steps
            for _, _, _, plan in pairs:
                if plan is not None:
                    plan.close()
        ratio = float(np.mean([a / b for a, b in pair_losses(net, held)]))
        ratio_op = [a / b for a, b in pair_losses(net, held, operator=True)]
        log(f"held-out pairs: mean |c - t| / |t| = {ratio:.4f}; mean |A (c - t)| / |A t| = "
            f"{np.mean(ratio_op):.4f} (before training {np.mean(before):.4f}; 1 = no gain)")
        params = net.get_params()
        np.savez(args.out, params=params, loss=np.array(hist), heldout_ratio=ratio,
                 heldout_op_ratio=float(np.mean(ratio_op)), heldout_op_ratios=np.array(ratio_op),
                 heldout_op_ratio_before=float(np.mean(before)), train_seconds=secs, loss_kind=args.loss,
                 n=args.n, problems=args.problems, iters=args.iters, steps=steps, seed=args.seed,
                 pairs=args.problems * args.iters, streamed=args.stream, lr=args.lr,
                 init=args.init or "seeded initialisation")
        seen = set()
        for _, _, _, plan in held:
            if plan is not None and id(plan) not in seen:
                seen.add(id(plan))
                plan.close()
        res = solve_compare(WORKLOADS["dns-128"], params, log)
        print(json.dumps({"loss": args.loss, "train_seconds": round(secs, 2), "heldout_ratio": ratio,
                          "heldout_op_ratio": [round(x, 4) for x in ratio_op],
                          "final_loss": hist[-1][1], "dns-128": res}), flush=True)
    elif args.cmd == "eval":
        params = np.load(args.weights)["params"]
        res = solve_compare(WORKLOADS[args.workload], params, log)
        print(json.dumps(res))
    else:
        w = WORKLOADS[args.workload]
        dims = (w.n, w.n + 2, w.n + 2) if w.bc == BC else (w.n,) * 3
        f_s, f_tf = speed(dims)
        t_s, t_tf = speed(dims, train=True)
        print(json.dumps({"dims": dims, "forward_s": f_s, "forward_tflops": f_tf,
                          "train_step_s": t_s, "train_tflops": t_tf,
                          "forward_flops": net_flops(dims)}))


if __name__ == "__main__":
    main()
