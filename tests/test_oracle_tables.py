"""Reproduction of the paper's printed results by the oracle (no GPU).

Error columns of Tables 2, 3 and 5 are exact pins (to the three printed
digits); SKS iteration counts are exact pins; GMRES counts are soft pins
(+-2), because the printed GMRES counts come from a left-preconditioned
library routine while the method is stated with right preconditioning.

Err2 ("the preconditioner used as a solver") does not state its right-hand
side.  Table 3's values are reproduced by A_p^{-1} F (F the sixth-order
right-hand side), Tables 2 and 5's by A_p^{-1} applied to the second-order
right-hand side h^2 f (with the Dirichlet data moved to it); each test uses
the reading its table fixes.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.onedim import OneD
from manufactured import source, table3_u, table5_u

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def close(a, b, rtol=0.015):
    return abs(a - b) <= rtol * abs(b)


def test_table2_one_dimensional():
    t = GOLD["table2"]
    k = 20.0
    w = k * math.pi
    u = lambda x: x * (1 - x) * np.cos(w * x)
    f = lambda x: -(2 + k * k * (math.pi ** 2 - 1) * x * (1 - x)) * np.cos(w * x) \
        + 2 * k * math.pi * (2 * x - 1) * np.sin(w * x)
    # f'' from the closed form of f (its second derivative, written out)
    def f2(x):
        p = x * (1 - x)
        c, s = np.cos(w * x), np.sin(w * x)
        g = -(2 + k * k * (math.pi ** 2 - 1) * p)        # coefficient of cos
        g1 = -k * k * (math.pi ** 2 - 1) * (1 - 2 * x)
        g2 = 2 * k * k * (math.pi ** 2 - 1)
        q = 2 * k * math.pi * (2 * x - 1)                 # coefficient of sin
        q1 = 4 * k * math.pi
        return (g2 * c - 2 * g1 * w * s - g * w * w * c) + (2 * q1 * w * c - q * w * w * s)
    eps_first = []
    for i, N in enumerate(t["n"]):
        m = OneD(N, k)
        F = m.rhs(f, f2)
        U, info = oracle.gmres(m.apply_A, m.apply_Pinv, F, restart=50, tol=1e-10)
        Us, infs = oracle.sks(m.apply_A, m.apply_Pinv, F, tol=1e-10)
        e6 = np.abs(Us - u(m.x)).max()
        e6g = np.abs(U - u(m.x)).max()
        e2 = np.abs(m.apply_Pinv(m.h ** 2 * f(m.x)) - u(m.x)).max()
        assert close(e6, t["err6"][i]), (N, e6)
        assert close(e6g, t["err6"][i], 0.05), (N, e6g)
        assert close(e2, t["err2"][i], 0.05), (N, e2)
        assert infs.iters == t["sks"][i]
        assert abs(info.iters - t["gmres"][i]) <= 2
        eps_first.append(infs.history[1] / infs.history[0])
    psi = oracle.psi_order(eps_first[-1], eps_first[-2], 2.0)
    assert abs(psi - t["psi"]) < 0.1


def test_theorem3_eigenvalues_1d():
    m = OneD(40, 7.0)
    A = np.diag(np.full(40, m.d2)) + m.d1 * (np.eye(40, k=1) + np.eye(40, k=-1))
    ev = np.sort(np.linalg.eigvalsh(A.real))
    assert np.allclose(ev, np.sort(m.eigenvalues().real), atol=1e-13)


def _table3d(ufun, bc, H, dirichlet_top, err2_second_order_rhs):
    k = 20.0
    prob = oracle.Problem.cube(H - 1, k, bc)
    u = ufun(k)
    f = source(u, k)
    F = oracle.rhs(prob, f, dirichlet_z=(None, u) if dirichlet_top else (None, None))
    ex = u.deriv(prob.points(), (0, 0, 0))
    U, info = oracle.solve(prob, F, "gmres", tol=1e-10)
    Us, infs = oracle.solve(prob, F, "sks", tol=1e-10)
    if err2_second_order_rhs:
        g = prob.h ** 2 * f.deriv(prob.points(), (0, 0, 0))
        if dirichlet_top:
            x, y, _ = prob.points()
            g[-1] -= u.deriv((x, y, np.array([1.0])), (0, 0, 0))[0]
    else:
        g = F
    return (np.abs(U - ex).max(), np.abs(oracle.apply_Pinv(prob, g) - ex).max(),
            info.iters, infs.iters, np.abs(Us - ex).max())


@pytest.mark.parametrize("i", [0, pytest.param(1, marks=pytest.mark.slow)])
def test_table3_dirichlet(i):
    t = GOLD["table3"]
    e6, e2, ng, ns, e6s = _table3d(table3_u, "DDDDDD", t["h"][i], False, False)
    assert close(e6, t["err6"][i]) and close(e6s, t["err6"][i])
    assert close(e2, t["err2"][i])
    assert ns == t["sks"][i]
    assert abs(ng - t["gmres"][i]) <= 2


@pytest.mark.parametrize("i", [0, pytest.param(1, marks=pytest.mark.slow)])
def test_table5_dirichlet_neumann(i):
    t = GOLD["table5"]
    e6, e2, ng, ns, e6s = _table3d(table5_u, "DDDDND", t["h"][i], True, True)
    assert close(e6, t["err6"][i]) and close(e6s, t["err6"][i])
    assert close(e2, t["err2"][i])
    assert ns == t["sks"][i]
    assert abs(ng - t["gmres"][i]) <= 2


@pytest.mark.parametrize("ki", range(5))
def test_table4_counts_h64(ki):
    """Table 4, h = 1/64: SKS exact or 'div' (None); GMRES no more than 2 above the
    printed count (the printed counts are left-preconditioned; for the hardest case,
    k = 50, right preconditioning needs markedly fewer steps)."""
    t = GOLD["table4"]
    k = float(t["k"][ki])
    g, s = t["rows"]["64"][ki]
    prob = oracle.Problem.cube(63, k)
    u = table3_u(k)
    F = oracle.rhs(prob, source(u, k))
    _, info = oracle.solve(prob, F, "gmres", tol=1e-10, maxit=100)
    _, infs = oracle.solve(prob, F, "sks", tol=1e-10, maxit=100)
    assert info.iters <= g + 2, info.iters
    if k <= 40:
        assert abs(info.iters - g) <= 2, info.iters
    if s is None:
        assert infs.status == "diverged"
    else:
        assert infs.iters == s
