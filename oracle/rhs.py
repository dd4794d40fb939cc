"""Right-hand side F of the h^2-scaled discrete system A U = F.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.

Interior part, right-hand side of eq. (scheme) times h^2 (Section 3.1):

  F = h^2 [ c_K f + (h^2/12)(1 - kappa/30) lap f + (h^4/360) lap^2 f
            + (h^4/180)(f_xxyy + f_xxzz + f_yyzz) ]

The mixed-derivative coefficient is read as h^4/180 rather than the printed
h^4/90: only h^4/180 makes the scheme consistent to sixth order (the symbol
check in the tests), and it reproduces the errors printed in Table 3.

Face terms (the source parts of the ghost relations, moved to the right):

* Neumann face at the low end of an axis n with tangential axes t1, t2,
  eq. (3DN) with beta = 0:  F += 2 h R_N,
    R_N = (h^2/6)(1 - kappa/20) f_n + (h^4/120) f_nnn + (7 h^4/360)(f_n t1t1 + f_n t2t2).
  The sign of the last term follows the derivation that precedes (3DN)
  (its printed +7h^5/180 is read as -7h^5/180: with the printed sign the
  ghost relation is only fifth-order accurate).  At the high end the normal
  derivative changes sign, so F -= 2 h R_N there.
* Sommerfeld face at z = 0, eqs. (3DIMP) and (3DDISCS):
    F += e^{ikh} mu3 [ 2 h Fbar + mu1 (h^5/3) Lbar ],
    Fbar = (h^2/6 + k^2 h^4/45) fbar_z - (i k h^4/90) fbar_zz + (h^4/120)(fbar_zzz - Lbar),
    Lbar = fbar_xxz + fbar_yyz,  fbar = e^{ikz} f.
  At z = top the same holds in the reflected coordinate z' = top - z.
* Nonhomogeneous Dirichlet data g on a z face (used for Table 5): the row
  next to the face holds G g (the h^2-scaled plane coupling), so F -= G g.
* Neumann data beta = du/dn (n the face's axis, derivative along +n) on a
  Neumann face, eq. (3DN): the ghost relation carries, besides -2h R_N,
    -2h B,  B = (1 - kappa/6 + kappa^2/120) beta
                - (h^4/180)(beta_t1t1t2t2 + beta_t1t1t1t1 + beta_t2t2t2t2)
                - (k^2 h^4/180)(beta_t1t1 + beta_t2t2),
  so F += 2h B on the low face and F -= 2h B on the high face (as R_N).

Edges and corners where several such faces meet receive the terms of every
face independently.
"""
from __future__ import annotations

import math

import numpy as np

from .functions import Separable
from .grid import Problem
from .scheme import apply_G_plane, coefficients


def _face_points(prob: Problem, ax: int, side: int):
    pts = list(prob.points())
    pts[ax] = np.array([0.0 if side == 0 else prob.length(ax)])
    return tuple(pts)


def interior_rhs(prob: Problem, f: Separable) -> np.ndarray:
    h, kap = prob.h, prob.kappa
    pts = prob.points()
    D = lambda a, b, c: f.deriv(pts, (a, b, c))
    cK = 1.0 - kap / 12.0 + kap * kap / 360.0
    lap = D(2, 0, 0) + D(0, 2, 0) + D(0, 0, 2)
    mixed = D(2, 2, 0) + D(2, 0, 2) + D(0, 2, 2)
    bilap = D(4, 0, 0) + D(0, 4, 0) + D(0, 0, 4) + 2.0 * mixed
    return h * h * (cK * D(0, 0, 0) + (h * h / 12.0) * (1.0 - kap / 30.0) * lap
                    + (h ** 4 / 360.0) * bilap + (h ** 4 / 180.0) * mixed)


def _neumann_RN(prob: Problem, f: Separable, ax: int, side: int) -> np.ndarray:
    """R_N on the face (derivatives taken along +axis), shape of the face plane."""
    h, kap = prob.h, prob.kappa
    pts = _face_points(prob, ax, side)
    t1, t2 = [a for a in range(3) if a != ax]

    def D(n_ax, n_t1=0, n_t2=0):
        o = [0, 0, 0]
        o[ax], o[t1], o[t2] = n_ax, n_t1, n_t2
        return f.deriv(pts, tuple(o))

    return ((h * h / 6.0) * (1.0 - kap / 20.0) * D(1) + (h ** 4 / 120.0) * D(3)
            + (7.0 * h ** 4 / 360.0) * (D(1, 2, 0) + D(1, 0, 2)))


def _neumann_data_term(prob: Problem, g: Separable, ax: int, side: int) -> np.ndarray:
    """B of eq. (3DN) for Neumann data beta = g on the face (tangential
    derivatives of g taken on the face plane)."""
    h, kap = prob.h, prob.kappa
    pts = _face_points(prob, ax, side)
    t1, t2 = [a for a in range(3) if a != ax]

    def D(n1, n2):
        o = [0, 0, 0]
        o[t1], o[t2] = n1, n2
        return g.deriv(pts, tuple(o))

    return ((1.0 - kap / 6.0 + kap * kap / 120.0) * D(0, 0)
            - (h ** 4 / 180.0) * (D(2, 2) + D(4, 0) + D(0, 4))
            - (prob.k ** 2 * h ** 4 / 180.0) * (D(2, 0) + D(0, 2)))


def _sommerfeld_term(prob: Problem, f: Separable, side: int) -> np.ndarray:
    """e^{ikh} mu3 [2h Fbar + mu1 h^5/3 Lbar] on a z face (reflected at the top)."""
    h, k = prob.h, prob.k
    c = coefficients(prob)
    pts = _face_points(prob, 2, side)
    sgn = 1.0 if side == 0 else -1.0   # d/dz' = sgn * d/dz
    ik = 1j * k

    def Dz(nz, nx=0, ny=0):
        return f.deriv(pts, (nx, ny, nz)) * (sgn ** nz)

    def fbar(m, nx=0, ny=0):
        # d^m/dz'^m (e^{ikz'} f) at z' = 0, Leibniz rule
        return sum(math.comb(m, j) * ik ** (m - j) * Dz(j, nx, ny) for j in range(m + 1))

    Lbar = fbar(1, 2, 0) + fbar(1, 0, 2)
    Fbar = ((h * h / 6.0 + k * k * h ** 4 / 45.0) * fbar(1) - (ik * h ** 4 / 90.0) * fbar(2)
            + (h ** 4 / 120.0) * (fbar(3) - Lbar))
    return c["e1"] * c["mu3"] * (2.0 * h * Fbar + c["mu1"] * (h ** 5 / 3.0) * Lbar)


def _add_face(F: np.ndarray, ax: int, side: int, term: np.ndarray):
    """Add a face plane term (shape with a length-1 ax dimension) to F."""
    arr_axis = 2 - ax
    idx = [slice(None)] * 3
    idx[arr_axis] = slice(0, 1) if side == 0 else slice(F.shape[arr_axis] - 1, None)
    F[tuple(idx)] += term


def rhs(prob: Problem, f: Separable, dirichlet_z=(None, None), neumann=None) -> np.ndarray:
    """F for source f; dirichlet_z = optional data g (Separable) on the z faces;
    neumann = optional {face index 0..5 (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi):
    Separable whose values on that face are beta = du/dn (along +axis)}."""
    F = interior_rhs(prob, f)
    h = prob.h
    for ax in range(3):
        for side in (0, 1):
            code = prob.bc[2 * ax + side]
            if code == "N":
                RN = _neumann_RN(prob, f, ax, side)
                _add_face(F, ax, side, (2.0 * h if side == 0 else -2.0 * h) * RN)
            elif code == "S":
                _add_face(F, ax, side, _sommerfeld_term(prob, f, side))
    for face, g in (neumann or {}).items():
        ax, side = divmod(face, 2)
        if prob.bc[face] != "N":
            raise ValueError("Neumann data given on a non-Neumann face")
        _add_face(F, ax, side, (2.0 * h if side == 0 else -2.0 * h) * _neumann_data_term(prob, g, ax, side))
    for side, g in enumerate(dirichlet_z):
        if g is None:
            continue
        if prob.bc[4 + side] != "D":
            raise ValueError("Dirichlet data given on a non-Dirichlet face")
        pts = _face_points(prob, 2, side)
        plane = g.deriv(pts, (0, 0, 0))[0]
        row = 0 if side == 0 else -1
        F[row] -= apply_G_plane(prob, plane)
    return F
