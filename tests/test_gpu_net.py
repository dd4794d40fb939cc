"""GPU parity of the learned correction network (include/h6net.h) against the
oracle (oracle/unet.py), and its use inside flexible GMRES.

Two comparisons:

* Against the oracle in BF16 storage mode (store=unet.round_bf16: values
  rounded to BF16 exactly where the network's definition stores BF16, every
  ReLU decided on the stored values, FP64 arithmetic otherwise), element by
  element: per weight block max |g_gpu - g_orc| / max |g_orc|.  What is left
  is the accumulation order: FP32 on the matrix cores against FP64 (relative
  2^-24 per term, about 1e-7 for a sum), which moves a stored value by one
  BF16 unit (2^-8 relative) only where it straddles a rounding boundary, and
  a ReLU only where the pre-activation is within that accumulation error of
  zero.  The bound is 2e-2 of the block's largest entry (about five BF16
  units), in both ReLU regimes.  Measured on gfx950: 1e-7 (forward) and
  4e-6 to 3e-3 (gradients) at 12 x 10 x 9, where nearly every stored value
  agrees bit for bit; 6e-3 (forward) and 8e-4 to 8e-3 (gradients) at
  80 x 64 x 56.
* Against the exact FP64 oracle (store=None) in relative 2-norm, which
  measures the BF16 model error itself: the 11 layers' outputs each rounded
  to BF16 (unit roundoff 2^-9) give about sqrt(11) 2^-9 = 0.7% forward and
  twice as many roundings backward; 3% is allowed when every ReLU is active.
  With mixed signs a pre-activation within the BF16 rounding error of zero
  can switch its ReLU on one side only, which moves a gradient block by
  about the square root of the switched fraction: 8% is allowed there
  (measured 5.8% at 12 x 10 x 9, 0.2% at 80 x 64 x 56; the element-wise
  comparison above is the tight one).

The gradient cases run at 12 x 10 x 9 and at 80 x 64 x 56 unknowns, where
the weight-gradient kernels grid-stride: 1,120 blocks of 16 x 4 x 4 voxels
at level 1 for the 512 workgroups of the tiled kernel (each walks at least
two), 560 tiles of 64 voxels at level 2 and 70 at level 3 for the 64
workgroup rows of the one-tap kernel."""
import numpy as np
import pytest
import torch

from oracle import unet
from paper_1212_1397_amd.workloads import init_net_params, random_field

pytestmark = pytest.mark.gpu

KH = 0.35
BIG = (80, 64, 56)


def params_for_test(seed=5, out_scale=1.0, bias=None, wscale=1.0):
    """Initial weights (seeded) with random biases, or all biases = `bias`."""
    p = init_net_params([(l[0], l[1], l[2]) for l in unet.LAYERS], seed)
    rng = np.random.default_rng(seed + 1)
    for name in p:
        W, b = p[name]
        W = W * (out_scale if name == "out" else wscale)
        b = 0.05 * rng.standard_normal(b.shape) if bias is None else np.full(b.shape, bias)
        p[name] = (W, b)
    return p


def oracle_params(p):
    """The weights as the device uses them (BF16); biases stay FP32 on the device."""
    return {k: (unet.round_bf16(W), np.asarray(b, dtype=np.float32).astype(np.float64)) for k, (W, b) in p.items()}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def maxrel(a, b):
    """max |a - b| / max |b| (element by element, scaled by the block's largest entry)."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_grads(h6, g, ref_store, ref_exact, tol_elem, tol_norm):
    gg = h6.unpack_net_params(g)
    worst = 0.0
    for name, _, _, _ in unet.LAYERS:
        eW, eb = maxrel(gg[name][0], ref_store[name][0]), maxrel(gg[name][1], ref_store[name][1])
        nW, nb = rel(gg[name][0], ref_exact[name][0]), rel(gg[name][1], ref_exact[name][1])
        print(f"  {name}: element-wise vs BF16-storage oracle dW {eW:.2e} db {eb:.2e}; "
              f"2-norm vs FP64 oracle dW {nW:.2e} db {nb:.2e}", flush=True)
        worst = max(worst, eW, eb)
        assert eW < tol_elem and eb < tol_elem, name
        assert nW < tol_norm and nb < tol_norm, name
    return worst


@pytest.fixture(scope="module")
def h6():
    from paper_1212_1397_amd import helmholtz6
    return helmholtz6


@pytest.mark.parametrize("dims", [(12, 10, 9), (17, 8, 6), BIG])
def test_forward_matches_oracle(h6, dims):
    p = params_for_test(out_scale=100.0)
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(p))
    shape = (dims[2], dims[1], dims[0])
    r = random_field(shape, 3)
    c = net.forward(torch.from_numpy(r).cuda(), KH).cpu().numpy()
    ref = unet.correction(oracle_params(p), r, KH, 1.0)     # k h passed as k = KH, h = 1
    ref_st = unet.correction(oracle_params(p), r, KH, 1.0, store=unet.round_bf16)
    print(f"dims {dims}: forward rel err {rel(c, ref):.2e} (FP64 oracle), element-wise "
          f"{maxrel(c, ref_st):.2e} (BF16-storage oracle)", flush=True)
    assert rel(c, ref) < 3e-2
    assert maxrel(c, ref_st) < 2e-2


def test_forward_is_homogeneous_and_zero_safe(h6):
    dims = (10, 9, 8)
    p = params_for_test(out_scale=100.0)
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(p))
    r = torch.from_numpy(random_field((8, 9, 10), 4)).cuda()
    c1 = net.forward(r, KH)
    c2 = net.forward(2.0 * r, KH)
    assert torch.equal(c2, 2.0 * c1)
    z = net.forward(torch.zeros_like(r), KH)
    assert torch.count_nonzero(z) == 0


@pytest.mark.parametrize("dims", [(17, 8, 6), BIG])
def test_inference_forward_equals_training_forward(h6, dims):
    """Inference forms the input features inside the first convolution, takes
    the encoder's pools from the convolution epilogues and reads the
    decoder's upsampled inputs on the fly; training materialises all three
    (its weight gradients need them).  Both compute the same values in the
    same order, so the training call's loss L = sum |c - t|^2 / sum |t|^2
    (FP64 sums over its own forward output) equals the loss of the inference
    output up to the rounding of those sums.  Odd grid sizes exercise the
    pools' missing children."""
    p = params_for_test(out_scale=100.0)
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(p))
    shape = (dims[2], dims[1], dims[0])
    r = random_field(shape, 13)
    t = random_field(shape, 14)
    c = net.forward(torch.from_numpy(r).cuda(), KH).cpu().numpy()
    loss, _ = net.gradients(torch.from_numpy(r).cuda(), KH, torch.from_numpy(t).cuda())
    host = float(np.sum(np.abs(c - t) ** 2) / np.sum(np.abs(t) ** 2))
    print(f"dims {dims}: training loss {loss:.15e}, from the inference output {host:.15e}", flush=True)
    assert abs(loss - host) <= 1e-12 * host


@pytest.mark.parametrize("dims", [(12, 10, 9), BIG])
@pytest.mark.parametrize("regime", ["active", "mixed"])
def test_gradients_match_oracle(h6, regime, dims):
    if regime == "active":
        p, tol = params_for_test(out_scale=100.0, bias=1.0, wscale=0.3), 3e-2
    else:
        p, tol = params_for_test(out_scale=100.0), 8e-2
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(p))
    shape = (dims[2], dims[1], dims[0])
    r = random_field(shape, 6)
    t = 0.3 * random_field(shape, 7)
    print(f"gradients {regime} dims {dims}", flush=True)
    loss, g = net.gradients(torch.from_numpy(r).cuda(), KH, torch.from_numpy(t).cuda())
    L_ref, grads = unet.loss_and_grads(oracle_params(p), r, KH, 1.0, t)
    L_st, grads_st = unet.loss_and_grads(oracle_params(p), r, KH, 1.0, t, store=unet.round_bf16)
    print(f"{regime}: loss gpu {loss:.6e} oracle {L_ref:.6e} (BF16 storage {L_st:.6e})", flush=True)
    assert abs(loss - L_ref) / L_ref < 1e-2
    assert abs(loss - L_st) / L_st < 1e-4
    worst = check_grads(h6, g, grads_st, grads, 2e-2, tol)
    print(f"{regime} {dims}: worst element-wise gradient difference {worst:.2e}", flush=True)


@pytest.mark.parametrize("bc,precision,n", [("DDDDDD", "fp64", (12, 10, 9)), ("DDNNSS", "mixed", (12, 10, 9)),
                                            ("DDNNSS", "mixed", (80, 62, 54))])
def test_operator_gradients_match_oracle(h6, bc, precision, n):
    """Operator-weighted loss |A (c - t)|^2 / |A t|^2: loss and gradients
    against the oracle with its own A (the gradient uses conj(A conj(.)) on
    both sides, so the comparison holds for every face type)."""
    import oracle
    h, k = 1.0 / (n[0] + 1), 30.0 + 0.3j
    p = params_for_test(out_scale=100.0, bias=1.0, wscale=0.3)
    plan = h6.Plan(n, h, k, bc, precision=precision)
    dims = plan.dims
    net = h6.Net(dims)
    net.set_params(h6.pack_net_params(p))
    shape = (dims[2], dims[1], dims[0])
    r = random_field(shape, 6)
    t = 0.3 * random_field(shape, 7)
    prob = oracle.Problem(n, h, k, tuple(bc))
    assert prob.shape == shape
    A = lambda v: oracle.apply_A(prob, v)
    print(f"operator gradients {bc} dims {dims}", flush=True)
    loss, g = net.gradients_op(plan, torch.from_numpy(r).cuda(), torch.from_numpy(t).cuda())
    L_ref, grads = unet.loss_and_grads_op(oracle_params(p), r, k, h, t, A)
    L_st, grads_st = unet.loss_and_grads_op(oracle_params(p), r, k, h, t, A, store=unet.round_bf16)
    print(f"{bc}: op loss gpu {loss:.6e} oracle {L_ref:.6e} (BF16 storage {L_st:.6e})", flush=True)
    assert abs(loss - L_ref) / L_ref < 1e-2
    assert abs(loss - L_st) / L_st < 1e-4
    check_grads(h6, g, grads_st, grads, 2e-2, 3e-2)
    l0 = net.train_step_op(plan, torch.from_numpy(r).cuda(), torch.from_numpy(t).cuda(), 1e-3)
    assert abs(l0 - loss) / loss < 1e-6
    other = h6.Net((dims[0] + 1, dims[1], dims[2]))
    z = torch.zeros(other.shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(h6.H6Error):
        other.gradients_op(plan, z, z)


def test_adam_step_and_loss_decrease(h6):
    dims = (12, 10, 9)
    p = params_for_test(out_scale=100.0)
    net = h6.Net(dims)
    flat0 = h6.pack_net_params(p)
    net.set_params(flat0)
    shape = (dims[2], dims[1], dims[0])
    r = torch.from_numpy(random_field(shape, 8)).cuda()
    t = torch.from_numpy(0.3 * random_field(shape, 9)).cuda()
    _, g = net.gradients(r, KH, t)
    lr = 1e-3
    loss0 = net.train_step(r, KH, t, lr)
    flat1 = net.get_params()
    # first Adam step from zero moments: w - lr g / (|g| + eps) (FP32 arithmetic)
    g32 = g.astype(np.float32)
    expect = flat0 - np.float32(lr) * g32 / (np.abs(g32) + np.float32(1e-8))
    np.testing.assert_allclose(flat1, expect, rtol=1e-5, atol=1e-6)
    losses = [loss0] + [net.train_step(r, KH, t, lr) for _ in range(20)]
    print("losses", [f"{x:.4f}" for x in losses[::5]], flush=True)
    assert losses[-1] < 0.9 * losses[0]


def test_learned_fgmres_converges_and_falls_back(h6):
    from paper_1212_1397_amd.workloads import WORKLOADS, gaussian_sources
    w = WORKLOADS["dns-128"]
    plan = h6.Plan(w.n, w.h, w.k, w.bc, precision="mixed")
    F = plan.rhs_gaussians(*gaussian_sources(w))
    U0, info0 = plan.solve(F, method="fgmres", restart=w.restart, tol=w.tol, maxit=300)
    assert info0["status"] == "ok"
    net = h6.Net(plan.dims)
    # a zero correction passes the acceptance test: every step uses it and the iterates
    # are those of the plain solve, bit for bit
    net.set_params(np.zeros(net.count, dtype=np.float32))
    plan.attach_net(net)
    U1, info1 = plan.solve(F, method="fgmres", restart=w.restart, tol=w.tol, maxit=300)
    print(f"plain {info0['iters']} its, zero correction {info1['iters']} its "
          f"({plan.learned_steps()} with the correction)", flush=True)
    assert plan.learned_steps() == info1["iters"] == info0["iters"]
    assert torch.equal(U1, U0)
    # a small random correction: the solve still converges to the tolerance
    net.set_params(h6.pack_net_params(params_for_test(out_scale=1.0)))
    U1, info1 = plan.solve(F, method="fgmres", restart=w.restart, tol=w.tol, maxit=300)
    assert info1["status"] == "ok" and info1["rel_resid"] <= w.tol
    assert float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0)) < 1e-6
    # a grossly wrong correction is rejected by the acceptance test: plain iterations
    net.set_params(h6.pack_net_params(params_for_test(out_scale=1e5)))
    U2, info2 = plan.solve(F, method="fgmres", restart=w.restart, tol=w.tol, maxit=300)
    assert plan.learned_steps() == 0
    assert info2["iters"] == info0["iters"] and info2["status"] == "ok"
    plan.attach_net(None)


def test_committed_weights_gain(h6):
    """What the trained network (paper_1212_1397_amd/data/net_dns128.npz)
    gains over the plain preconditioner, as it comes out: on fresh pairs
    (residual, target) of a held-out 128^3 problem the corrected
    preconditioner's residual |A (c - t)| against the plain one's |A t| (the
    quantity the solver's acceptance test compares), and mixed FGMRES(30) on the
    128 x 130 x 130 workload with and without the correction."""
    import os
    from paper_1212_1397_amd import learned
    from paper_1212_1397_amd.workloads import WORKLOADS
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1212_1397_amd", "data", "net_dns128.npz")
    params = np.load(path)["params"]
    pairs = learned.make_pairs(128, 1, 4, seed=424_242, log=lambda m: None, keep_plans=True)
    net = h6.Net(tuple(pairs[0][0].shape[::-1]))
    net.set_params(params)
    ratios = [a / b for a, b in learned.pair_losses(net, pairs, operator=True)]
    for _, _, _, plan in pairs[:1]:
        plan.close()
    print(f"held-out residual ratios |A (c - t)| / |A t|: {[round(x, 4) for x in ratios]}", flush=True)
    res = learned.solve_compare(WORKLOADS["dns-128"], params, log=lambda m: None)
    print(f"dns-128 mixed FGMRES(30): plain {res['plain']['iters']} steps, learned "
          f"{res['learned']['iters']} steps ({res['learned']['steps_with_correction']} with the "
          f"correction), solution difference {res['solution_rel_diff']:.2e}", flush=True)
    # the network lowers the preconditioner's residual on held-out pairs, the
    # acceptance test takes it on every step, and the corrected solve needs fewer
    # steps than the plain one (measured: 9 against 10)
    assert float(np.mean(ratios)) < 1.0
    assert res["plain"]["rel_resid"] <= 1e-8 and res["learned"]["rel_resid"] <= 1e-8
    assert res["learned"]["steps_with_correction"] == res["learned"]["iters"]
    assert res["learned"]["iters"] < res["plain"]["iters"]
    assert res["solution_rel_diff"] < 1e-6


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-5)])
def test_training_pair_matches_oracle(h6, precision, tol):
    """h6net_training_pair: r = F - A U and t = (U* - U) - A_p^{-1} r against
    the oracle's operator and preconditioner (complex64 preconditioner
    arithmetic in mixed plans: relative error about 1e-6)."""
    import oracle
    n, h, k, bc = (20, 13, 17), 1.0 / 21, 7.0 + 0.2j, "DDNNSS"
    plan = h6.Plan(n, h, k, bc, precision=precision)
    prob = oracle.Problem(n, h, k, tuple(bc))
    F, Us, U = (random_field(prob.shape, s) for s in (21, 22, 23))
    r, t = plan.training_pair(*(torch.from_numpy(a).cuda() for a in (F, Us, U)))
    r_ref = F - oracle.apply_A(prob, U)
    t_ref = (Us - U) - oracle.apply_Pinv(prob, r_ref)
    er, et = maxrel(r.cpu().numpy(), r_ref), maxrel(t.cpu().numpy(), t_ref)
    print(f"{precision}: r error {er:.2e}, t error {et:.2e}", flush=True)
    assert er <= 1e-12 and et <= tol
