"""The chirp-z (Bluestein) transform path of A_p^{-1} (Section 3.3's sine /
cosine transforms for odd M = n + 1 <= 255) against the FP64 oracle.

Grids are chosen so that every combination the kernels specialise on runs:
sine and cosine bases, x lines and y columns, convolution length P = 256
(M <= 129, including M = 129 where P = 2M - 2 exactly) and P = 512
(131 <= M <= 255, including the longest line n' = 256), the smallest M = 3,
and FP64 and complex64 plans.  Bounds are
those of the other A_p^{-1} parity tests: 1e-12 relative in FP64, 5e-5 for the
complex64 preconditioner.  The same plans built with the dense transforms
(H6_DENSE_TRANSFORMS set at setup) must agree with the oracle too and must
not be bit-identical to the chirp-z results, which shows the switch took the
other path.  The chirp-z path is forced through the autotuner's cache file.
"""
import numpy as np
import pytest

import oracle
from paper_1212_1397_amd.workloads import random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _h6():
    from paper_1212_1397_amd import helmholtz6
    return helmholtz6


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def force_paths(plan, tmp_path, xfast, yfast):
    """Choose the transform path per axis (0 dense, 2 chirp-z) through the
    autotuner's cache file (the untuned default takes chirp-z only where its
    FFT length is nearly all signal)."""
    h6 = _h6()
    arch = torch.cuda.get_device_properties(0).gcnArchName
    nx, ny, nz = plan.dims
    path = tmp_path / f"tune_{nx}_{ny}_{nz}_{xfast}{yfast}.txt"
    path.write_text(f"h6tune3 {arch} {nx} {ny} {nz} {h6.PRECISIONS[plan.precision]} tz=16 xfast={xfast} "
                    f"yfast={yfast} xlines=4 ylines=16\n")
    plan.autotune(str(path))


CASES = [
    # x sine P = 512 (M = 201), y cosine P = 512 (M = 131)
    ((200, 130, 3), 20.0 + 0.3j, "DDNNSS"),
    # x cosine with the longest line (M = 255, n'x = 256), y sine P = 256 at M = 127
    ((254, 126, 2), 18.0, "NNDDDN"),
    # M = 129 on both axes: P = 256 = 2M - 2, no spare lag
    ((128, 128, 2), 25.0 + 0.2j, "DDNNSS"),
    # M = 3 and M = 5
    ((2, 4, 3), 3.0, "DDNNDD"),
    ((4, 2, 5), 2.5 + 0.5j, "NNDDSS"),
]


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("mixed", 5e-5)])
@pytest.mark.parametrize("n,k,bc", CASES)
def test_bluestein_pinv_parity(n, k, bc, prec, bound, tmp_path):
    h6 = _h6()
    prob = oracle.Problem(n, 1.0 / (max(n) + 1), complex(k), tuple(bc))
    x = random_field(prob.shape, seed=21)
    ref = oracle.apply_Pinv(prob, x)
    plan = h6.Plan(prob.n, prob.h, prob.k, bc, precision=prec)
    force_paths(plan, tmp_path, 2, 2)
    z = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    plan.close()
    assert relerr(z, ref) <= bound


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("mixed", 5e-5)])
def test_dense_switch_takes_the_other_path(monkeypatch, tmp_path, prec, bound):
    """H6_DENSE_TRANSFORMS at setup builds no chirp-z tables: a cache line
    asking for chirp-z then falls back to the dense product, which differs
    in rounding from the chirp-z result of a plan built without it."""
    h6 = _h6()
    n, k, bc = (200, 130, 3), 20.0 + 0.3j, "DDNNSS"
    prob = oracle.Problem(n, 1.0 / (max(n) + 1), complex(k), tuple(bc))
    x = random_field(prob.shape, seed=5)
    ref = oracle.apply_Pinv(prob, x)
    plan = h6.Plan(prob.n, prob.h, prob.k, bc, precision=prec)
    force_paths(plan, tmp_path, 2, 2)
    zb = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    plan.close()
    monkeypatch.setenv("H6_DENSE_TRANSFORMS", "1")
    plan = h6.Plan(prob.n, prob.h, prob.k, bc, precision=prec)
    force_paths(plan, tmp_path, 2, 2)
    zd = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    plan.close()
    assert relerr(zb, ref) <= bound
    assert relerr(zd, ref) <= bound
    assert not np.array_equal(zb, zd)


@pytest.mark.parametrize("M,default", [(129, 2), (127, 2), (121, 2), (119, 0), (97, 0), (255, 2), (241, 2),
                                       (239, 0), (201, 0), (3, 0)])
def test_untuned_default_path(tmp_path, M, default):
    """Untuned plans take chirp-z only where 2M - 2 >= 15/16 of its FFT
    length: the untuned result equals the forced choice of that path."""
    h6 = _h6()
    n = M - 1
    prob = oracle.Problem((n, 2, 2), 1.0 / (n + 1), 5.0 + 0.1j, tuple("DDDDDD"))
    x = random_field(prob.shape, seed=9)
    plan = h6.Plan(prob.n, prob.h, prob.k, "DDDDDD", precision="mixed")
    z0 = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    force_paths(plan, tmp_path, default, 0)
    z1 = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    force_paths(plan, tmp_path, 2 - default, 0)
    z2 = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    plan.close()
    assert np.array_equal(z0, z1)
    assert not np.array_equal(z0, z2)


def test_bluestein_solve_parity(tmp_path):
    """A whole FGMRES solve with the chirp-z transforms inside its graphs."""
    h6 = _h6()
    n, k, bc = (96, 64, 40), 16.0 + 0.2j, "DDNNSS"
    prob = oracle.Problem(n, 1.0 / 97, complex(k), tuple(bc))
    F = random_field(prob.shape, seed=8)
    plan = h6.Plan(prob.n, prob.h, prob.k, bc)
    force_paths(plan, tmp_path, 2, 2)
    U, info = plan.solve(to_gpu(F), method="fgmres", restart=30, tol=1e-11, maxit=400)
    assert info["status"] == "ok" and info["rel_resid"] <= 1e-11
    u = U.cpu().numpy()
    r = F - oracle.apply_A(prob, u)
    assert np.linalg.norm(r) / np.linalg.norm(F) <= 1.01e-11
    plan.close()


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("mixed", 5e-5)])
def test_autotuner_cache_selects_the_transform_path(tmp_path, prec, bound):
    """At 128^3 (M = 129 on both axes) the autotuner chooses per axis between
    the chirp-z path and the dense product; each of the four choices, forced
    through the cache file, agrees with the oracle, and the untuned plan
    (chirp-z on both axes) equals the (2, 2) choice bit for bit."""
    import os
    from paper_1212_1397_amd.workloads import WORKLOADS
    h6 = _h6()
    w = WORKLOADS["dns-128"]
    prob = oracle.Problem.cube(w.n, w.k, w.bc)
    plan = h6.Plan(w.n, w.h, w.k, w.bc, precision=prec)
    x = random_field(prob.shape, seed=2)
    ref = oracle.apply_Pinv(prob, x)
    z_def = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    arch = torch.cuda.get_device_properties(0).gcnArchName
    nx, ny, nz = plan.dims
    got = {}
    for xf, yf in [(0, 0), (2, 0), (0, 2), (2, 2)]:
        path = os.path.join(tmp_path, f"tune_{xf}{yf}.txt")
        with open(path, "w") as f:
            f.write(f"h6tune3 {arch} {nx} {ny} {nz} {h6.PRECISIONS[prec]} tz=16 xfast={xf} yfast={yf} "
                    f"xlines=4 ylines=16\n")
        plan.autotune(path)
        got[(xf, yf)] = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
        assert relerr(got[(xf, yf)], ref) <= bound, (xf, yf)
    plan.close()
    assert np.array_equal(got[(2, 2)], z_def)
    assert not np.array_equal(got[(0, 0)], z_def)


def test_bluestein_every_odd_M(tmp_path):
    """Every odd M = 3 .. 255 (both convolution lengths, every output-slot
    count of the post-processing) in the sine and the cosine basis on x,
    FP64, against the oracle."""
    h6 = _h6()
    worst = 0.0
    for M in range(3, 256, 2):
        for bc in ("DDDDDD", "NNDDDD"):
            prob = oracle.Problem((M - 1, 2, 2), 1.0 / M, 3.0 + 0.2j, tuple(bc))
            x = random_field(prob.shape, seed=M)
            plan = h6.Plan(prob.n, prob.h, prob.k, bc)
            force_paths(plan, tmp_path, 2, 0)
            z = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
            plan.close()
            e = relerr(z, oracle.apply_Pinv(prob, x))
            worst = max(worst, e)
            assert e <= 1e-12, (M, bc, e)
    print(f"worst relative error over odd M = 3..255: {worst:.1e}", flush=True)
