"""The pins above catch plausible mistakes: each test plants one mistake in the
oracle (on the CPU, through monkeypatching) and checks that a pin fails."""
import math

import numpy as np
import pytest

import importlib

import oracle

orhs = importlib.import_module("oracle.rhs")
oscheme = importlib.import_module("oracle.scheme")
from dense_assembly import dense_A
from manufactured import mixed_pattern_u, neumann_data_z_u, neumann_z_u, normal_derivative, source


def _ratio(bc, k, u, ns=(15, 31)):
    errs = []
    for n in ns:
        prob = oracle.Problem.cube(n, k, bc)
        F = oracle.rhs(prob, source(u, k))
        U, info = oracle.solve(prob, F, "gmres", tol=1e-13, maxit=300)
        errs.append(np.abs(U - u.deriv(prob.points(), (0, 0, 0))).max())
    return errs[0] / errs[1]


def test_neumann_sign_mistake_lowers_order(monkeypatch):
    good = _ratio("DDDDND", 10.0, neumann_z_u())
    orig = orhs._neumann_RN

    def flipped(prob, f, ax, side):
        h = prob.h
        pts = orhs._face_points(prob, ax, side)
        t1, t2 = [a for a in range(3) if a != ax]
        o1 = [0, 0, 0]; o1[ax] = 1; o1[t1] = 2
        o2 = [0, 0, 0]; o2[ax] = 1; o2[t2] = 2
        mixed = f.deriv(pts, tuple(o1)) + f.deriv(pts, tuple(o2))
        return orig(prob, f, ax, side) - 2 * (7.0 * h ** 4 / 360.0) * mixed

    monkeypatch.setattr(orhs, "_neumann_RN", flipped)
    bad = _ratio("DDDDND", 10.0, neumann_z_u())
    assert good > 55 and bad < 40, (good, bad)


def test_sommerfeld_mu1_term_dropped_lowers_order(monkeypatch):
    k = 10.0 + 0.1j
    u = mixed_pattern_u(k)
    good = _ratio("DDNNSS", k, u)
    orig = orhs._sommerfeld_term

    def dropped(prob, f, side):
        c = oracle.coefficients(prob)
        h = prob.h
        pts = orhs._face_points(prob, 2, side)
        sgn = 1.0 if side == 0 else -1.0
        ik = 1j * prob.k
        L = sum(ik ** (1 - j) * f.deriv(pts, (2, 0, j)) * sgn ** j for j in range(2)) \
            + sum(ik ** (1 - j) * f.deriv(pts, (0, 2, j)) * sgn ** j for j in range(2))
        return orig(prob, f, side) - c["e1"] * c["mu3"] * c["mu1"] * (h ** 5 / 3.0) * L

    monkeypatch.setattr(orhs, "_sommerfeld_term", dropped)
    bad = _ratio("DDNNSS", k, u)
    assert good > 45 and bad < 40, (good, bad)


def test_wrong_Q_coefficient_caught_by_row_assembly(monkeypatch):
    orig = oscheme.sommerfeld_QR

    def wrong(c):
        Q, R = orig(c)
        return (Q[0], Q[1] * 1.01, Q[2]), R

    monkeypatch.setattr(oscheme, "sommerfeld_QR", wrong)
    prob = oracle.Problem((3, 3, 3), 0.25, 6.0 + 0.5j, tuple("DDNNSS"))
    A = dense_A(prob)
    N = A.shape[0]
    cols = np.eye(N, dtype=np.complex128)
    Am = np.stack([oracle.apply_A(prob, cols[j].reshape(prob.shape)).ravel() for j in range(N)], 1)
    assert np.abs(A - Am).max() > 1e-4


def test_wrong_triple_product_sign_caught_by_eigenmodes(monkeypatch):
    orig = oscheme.coefficients

    def wrong(prob):
        c = orig(prob)
        c["b"] = -c["b"]
        return c

    monkeypatch.setattr(oscheme, "coefficients", wrong)
    prob = oracle.Problem.cube(7, 3.0)
    x, y, z = prob.points()
    v = (np.sin(3 * np.pi * z)[:, None, None] * np.sin(2 * np.pi * y)[None, :, None]
         * np.sin(5 * np.pi * x)[None, None, :]) + 0j
    lam = oracle.dirichlet_eigenvalue(prob, 5, 2, 3)
    assert np.abs(oracle.apply_A(prob, v) - lam * v).max() > 1e-6


def test_wrong_preconditioner_end_row_caught(monkeypatch):
    op = importlib.import_module("oracle.precond")
    orig = op.z_tridiagonal

    def wrong(prob):
        sub, diag, sup = orig(prob)
        sup = sup.copy()
        sup[0] = 1.0
        return sub, diag, sup

    monkeypatch.setattr(op, "z_tridiagonal", wrong)
    prob = oracle.Problem.cube(6, 5.0, "DDDDSS")
    rng = np.random.default_rng(0)
    r = rng.standard_normal(prob.shape) + 0j
    assert np.abs(oracle.apply_Ap(prob, oracle.apply_Pinv(prob, r)) - r).max() > 1e-3


def test_neumann_data_high_order_terms_dropped_lowers_order(monkeypatch):
    """Keeping only the leading beta term of eq. (3DN) (dropping its h^5/90
    tangential-derivative terms) leaves a fourth-order scheme."""
    u = neumann_data_z_u()

    def ratio():
        errs = []
        for n in (15, 31):
            prob = oracle.Problem.cube(n, 10.0, "DDDDND")
            F = oracle.rhs(prob, source(u, 10.0), neumann={4: normal_derivative(u, 2)})
            U, info = oracle.solve(prob, F, "gmres", tol=1e-13, maxit=300)
            errs.append(np.abs(U - u.deriv(prob.points(), (0, 0, 0))).max())
        return errs[0] / errs[1]

    good = ratio()

    def leading_only(prob, g, ax, side):
        kap = prob.kappa
        pts = orhs._face_points(prob, ax, side)
        return (1.0 - kap / 6.0 + kap * kap / 120.0) * g.deriv(pts, (0, 0, 0))

    monkeypatch.setattr(orhs, "_neumann_data_term", leading_only)
    bad = ratio()
    assert good > 55 and bad < 40, (good, bad)
