"""Mixed precision (complex64 preconditioner, FP64 operator / residual /
Arnoldi) against the FP64 CPU oracle.

Bounds: the preconditioner's transforms and z solves run in FP32 (unit
roundoff 6e-8); a few dozen rounding steps per value, amplified by the
conditioning of the near-resonant z systems (~1e2), give the 5e-5 relative
bound used for A_p^{-1}.  Solves stop on the true FP64 residual, so the
returned residual meets the tolerance exactly as in FP64; the solution is
compared with the oracle's FP64 solution at tol 1e-11, and the two differ by
at most (condition of A) x (residual gap) - measured ~1e-8 relative at tol
1e-8, bounded here by 1e-6.
"""
import numpy as np
import pytest

import oracle
from oracle.functions import gaussian_sources
from paper_1212_1397_amd.workloads import WORKLOADS, gaussian_sources as wl_sources, random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _h6():
    from paper_1212_1397_amd import helmholtz6
    return helmholtz6


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,k,bc", [((70, 37, 45), 11.0 + 0.3j, "DDNNSS"),
                                    ((256, 256, 3), 30.0 + 0.3j, "DDNNSS"),
                                    ((256, 256, 2), 25.0, "NNDDDN")])
def test_mixed_pinv_accuracy(n, k, bc):
    h6 = _h6()
    prob = oracle.Problem(n, 1.0 / (max(n) + 1), complex(k), tuple(bc))
    plan = h6.Plan(prob.n, prob.h, prob.k, bc, precision="mixed")
    x = random_field(prob.shape, seed=4)
    z = plan.apply_Pinv(to_gpu(x)).cpu().numpy()
    err = relerr(z, oracle.apply_Pinv(prob, x))
    assert err <= 5e-5, err
    # the operator stays FP64 in mixed plans
    assert relerr(plan.apply_A(to_gpu(x)).cpu().numpy(), oracle.apply_A(prob, x)) <= 1e-12


@pytest.mark.parametrize("method", ["fgmres", "sks"])
def test_mixed_solve_dns128(method):
    h6 = _h6()
    w = WORKLOADS["dns-128"]
    prob = oracle.Problem.cube(w.n, w.k, w.bc)
    centres, amps, sigma = wl_sources(w)
    F = oracle.rhs(prob, gaussian_sources(centres, amps, sigma))
    U_ref, info = oracle.solve(prob, F, "gmres", restart=30, tol=1e-11)
    plan = h6.Plan(w.n, w.h, w.k, w.bc, precision="mixed")
    U, gi = plan.solve(to_gpu(F), method=method, restart=30, tol=w.tol, maxit=200)
    assert gi["status"] == "ok" and gi["rel_resid"] <= w.tol
    Uc = U.cpu().numpy()
    r = F - oracle.apply_A(prob, Uc)
    assert np.linalg.norm(r) / np.linalg.norm(F) <= w.tol * 1.01
    assert relerr(Uc, U_ref) <= 1e-6


def test_mixed_rejects_plain_gmres():
    h6 = _h6()
    plan = h6.Plan(8, 1 / 9, 3.0, precision="mixed")
    F = to_gpu(random_field(plan.shape, 1))
    with pytest.raises(h6.H6Error) as e:
        plan.solve(F, method="gmres")
    assert e.value.status == -1
