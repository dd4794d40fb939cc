"""Sixth-order convergence of the scheme with each face closure, and second-order
convergence of the preconditioner used alone (no GPU).

Error ratios of successive grids (h = 1/16, 1/32, 1/64) must approach 2^6 = 64
for the discrete solution of A U = F and 2^2 = 4 for A_p^{-1} F.  A dropped
term or a wrong sign in the interior scheme, the right-hand side or any closure
lowers the observed order.
"""
import math

import numpy as np
import pytest

import oracle
from manufactured import (mixed_pattern_u, neumann_data_y_u, neumann_data_z_u, neumann_y_factor, neumann_z_u,
                          normal_derivative, source, sommerfeld_z_factor)
from oracle.functions import Separable, Sin, Term


def errors(bc, k, u, ns=(15, 31, 63), data_faces=()):
    e6, e2 = [], []
    for n in ns:
        prob = oracle.Problem.cube(n, k, bc)
        nd = {f: normal_derivative(u, f // 2) for f in data_faces}
        F = oracle.rhs(prob, source(u, k), neumann=nd)
        U, info = oracle.solve(prob, F, "gmres", tol=1e-13, maxit=300)
        assert info.status == "ok"
        ex = u.deriv(prob.points(), (0, 0, 0))
        e6.append(np.abs(U - ex).max())
        e2.append(np.abs(oracle.apply_Pinv(prob, F) - ex).max())
    r6 = [e6[i] / e6[i + 1] for i in range(len(e6) - 1)]
    r2 = [e2[i] / e2[i + 1] for i in range(len(e2) - 1)]
    return r6, r2


CASES = {
    "dirichlet": ("DDDDDD", 10.0, lambda k: Separable([Term(1.0, Sin(math.pi), Sin(2 * math.pi),
                                                             Sin(3 * math.pi) * sommerfeld_z_factor(2.0))]),
                  (58, 66)),
    "neumann_z": ("DDDDND", 10.0, lambda k: neumann_z_u(), (60, 70)),
    "neumann_y": ("DDNNDD", 10.0, lambda k: Separable([Term(1.0, Sin(math.pi), neumann_y_factor(),
                                                             Sin(2 * math.pi))]), (60, 70)),
    "sommerfeld_z": ("DDDDSS", 10.0 + 0.1j, lambda k: Separable([Term(1.0, Sin(math.pi), Sin(2 * math.pi),
                                                                     sommerfeld_z_factor(k))]), (58, 68)),
    "mixed_pattern": ("DDNNSS", 10.0 + 0.1j, mixed_pattern_u, (58, 68)),
}

# nonzero Neumann data (eq. (3DN)): beta = du/dn of the manufactured solution
DATA_CASES = {
    "neumann_data_z": ("DDDDND", 10.0, neumann_data_z_u, (4,)),
    "neumann_data_y": ("DDNNDD", 10.0, neumann_data_y_u, (2, 3)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sixth_order(name):
    bc, k, ufun, (lo, hi) = CASES[name]
    r6, r2 = errors(bc, k, ufun(k))
    assert lo <= r6[-1] <= hi, r6
    assert r6[0] > 40, r6
    assert all(3.6 <= r <= 4.4 for r in r2), r2


@pytest.mark.parametrize("name", list(DATA_CASES))
def test_sixth_order_with_neumann_data(name):
    bc, k, ufun, faces = DATA_CASES[name]
    r6, _ = errors(bc, k, ufun(), data_faces=faces)
    assert 58 <= r6[-1] <= 70 and r6[0] > 55, r6
