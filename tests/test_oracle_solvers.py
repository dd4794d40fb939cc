"""Oracle solvers against brute force, the paper's convergence bound and a
closed-form case (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from dense_assembly import dense_A
from oracle.functions import Separable, Sin, Term, gaussian_sources
from manufactured import source

BRUTE_CASES = [("DDDDDD", 5.0), ("DDNNSS", 6.0 + 0.4j), ("NNNNSS", 4.0 + 0.2j), ("DDDDND", 3.0),
               ("NNDDSD", 5.5 + 0.1j)]


@pytest.mark.parametrize("bc,k", BRUTE_CASES)
def test_solvers_match_dense_solve(bc, k):
    prob = oracle.Problem((6, 5, 7), 1.0 / 8.0, complex(k), tuple(bc))
    rng = np.random.default_rng(7)
    F = rng.standard_normal(prob.shape) + 1j * rng.standard_normal(prob.shape)
    U_ref = np.linalg.solve(dense_A(prob), F.ravel()).reshape(prob.shape)
    scale = np.abs(U_ref).max()
    for method in ("gmres", "fgmres"):
        U, info = oracle.solve(prob, F, method, restart=7, tol=1e-13, maxit=500)
        assert info.status == "ok"
        assert np.abs(U - U_ref).max() <= 1e-10 * scale
    U, info = oracle.solve(prob, F, "sks", tol=1e-13, maxit=500)
    if info.status == "ok":
        assert np.abs(U - U_ref).max() <= 1e-10 * scale
    Uc, infc = oracle.solve(prob, F, "sks_correction", tol=1e-13, maxit=500)
    assert infc.status == info.status
    if info.status == "ok":
        assert abs(infc.iters - info.iters) <= 1
        assert np.abs(Uc - U_ref).max() <= 1e-10 * scale


def test_restart_continues_to_tolerance():
    prob = oracle.Problem.cube(9, 12.0 + 0.1j, "DDNNSS")
    F = oracle.rhs(prob, gaussian_sources([(0.4, 0.5, 0.6)], [1.0], 0.1))
    U1, i1 = oracle.solve(prob, F, "gmres", restart=2, tol=1e-11, maxit=400)
    U2, i2 = oracle.solve(prob, F, "gmres", restart=40, tol=1e-11, maxit=400)
    assert i1.status == i2.status == "ok"
    assert i1.iters >= i2.iters
    r = F - oracle.apply_A(prob, U1)
    assert np.linalg.norm(r) / np.linalg.norm(F) <= 1e-11
    assert np.abs(U1 - U2).max() <= 1e-9 * np.abs(U2).max()


@pytest.mark.parametrize("k", [2.0, 4.5])
def test_corollary1_bound_dirichlet(k):
    """Section 3.4 (3Dest): Dirichlet faces and k^2 < 25 give ||r_n|| <= (3/4)^n ||r_0||,
    for SKS (whose iteration matrix has eigenvalues -d with |d| < 3/4 in a unitary
    eigenbasis) and hence for GMRES, which minimises the residual."""
    prob = oracle.Problem.cube(15, k)
    rng = np.random.default_rng(3)
    F = rng.standard_normal(prob.shape) + 1j * rng.standard_normal(prob.shape)
    _, info = oracle.solve(prob, F, "sks", tol=1e-12, maxit=60)
    for n, eps in enumerate(info.history, start=1):
        assert eps <= 0.75 ** n * (1 + 1e-12)
    _, ig = oracle.solve(prob, F, "gmres", restart=60, tol=1e-12, maxit=60)
    for n, eps in enumerate(ig.history, start=1):
        assert eps <= 0.75 ** n * (1 + 1e-12)


def test_single_mode_closed_form():
    """u = sin(pi x) sin(2 pi y) sin(3 pi z), all Dirichlet: F is proportional to the
    (1,2,3) discrete eigenmode, so U = F / lambda_123 and GMRES needs one step."""
    k = 10.0
    prob = oracle.Problem.cube(32, k)
    u = Separable([Term(1.0, Sin(math.pi), Sin(2 * math.pi), Sin(3 * math.pi))])
    F = oracle.rhs(prob, source(u, k))
    lam = oracle.dirichlet_eigenvalue(prob, 1, 2, 3)
    U, info = oracle.solve(prob, F, "gmres", restart=20, tol=1e-10)
    assert info.iters == 1 and info.status == "ok"
    assert np.abs(U - F / lam).max() <= 1e-12 * np.abs(U).max()
    ex = u.deriv(prob.points(), (0, 0, 0))
    assert np.abs(U - ex).max() < 1e-6


def test_sks_divergence_flagged():
    """Table 3 / Table 4 at h = 1/32, k = 20: SKS diverges."""
    from manufactured import table3_u
    prob = oracle.Problem.cube(31, 20.0)
    F = oracle.rhs(prob, source(table3_u(20.0), 20.0))
    _, info = oracle.solve(prob, F, "sks", tol=1e-10, maxit=200)
    assert info.status == "diverged"


def test_gaussian_factor_derivatives():
    """Hermite derivative formula against finite differences of lower orders."""
    from oracle.functions import Gauss
    g = Gauss(0.3, 0.07)
    x = np.linspace(0.1, 0.5, 11)
    e = 1e-5
    for m in range(1, 6):
        fd = (g.d(x + e, m - 1) - g.d(x - e, m - 1)) / (2 * e)
        assert np.allclose(g.d(x, m), fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())
