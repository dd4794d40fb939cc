"""The sixth-order compact 27-point operator A (h^2-scaled), matrix free.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.

Definition (Section 3.1, eq. (scheme), left-hand side multiplied by h^2, with
D_a = h^2 delta_a^2 and kappa = (k h)^2):

    A U = (D_x + D_y + D_z) U + (1/6)(1 + kappa/30)(D_x D_y + D_x D_z + D_y D_z) U
          + (1/30) D_x D_y D_z U + kappa (1 - kappa/12 + kappa^2/360) U.

This equals D_z G U + P U with the in-plane operators

    G = I + (1/6)(1 + kappa/30)(D_x + D_y) + (1/30) D_x D_y,
    P = D_x + D_y + (1/6)(1 + kappa/30) D_x D_y + kappa c_K I,  c_K = 1 - kappa/12 + kappa^2/360,

so row l of A U is G U_{l-1} - 2 G U_l + G U_{l+1} + P U_l.  G is exactly the
operator that multiplies the ghost plane in the boundary closures (3DN) and
(3DDISCS), which lets each z-face closure replace the single term G U_ghost:

* Dirichlet face: the boundary plane holds u = 0 (no unknowns there).
* Neumann face, eq. (3DN) with beta = 0: G U_{-1} = G U_1 - 2 h R_N, where
  R_N only holds source terms (moved to the right-hand side, oracle.rhs).
* Sommerfeld face, eq. (3DDISCS): G U_{-1} = Q U_1 + R U_0 - (source terms)
  with the complex in-plane operators Q and R given in ``sommerfeld_QR``.

Neumann faces on the x and y axes act through the mirror ghost U_{-1} = U_1
inside D_x and D_y wherever those appear (the in-plane analogue of (3DN)).
The top z face is the mirror image of the bottom one (end of Section 3.2.2).
"""
from __future__ import annotations

import cmath

import numpy as np

from .grid import Problem


def coefficients(prob: Problem) -> dict:
    """Scalar coefficients of G, P and of the Sommerfeld closure (Section 3)."""
    kap = prob.kappa
    kh = prob.k * prob.h
    ikh = 1j * kh
    a = (1.0 + kap / 30.0) / 6.0
    cK = 1.0 - kap / 12.0 + kap * kap / 360.0
    # mu_3 and mu_1 of Section 3.2.2 (the parameters that match (scheme)).
    mu3 = 1.0 / (1.0 + (2.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0))
    mu1 = (ikh / 90.0 + (1.0 + kap / 30.0) / (6.0 * mu3)) / (1.0 + 2.0 * ikh / 3.0)
    e1 = cmath.exp(ikh)
    e2 = cmath.exp(2.0 * ikh)
    return dict(kappa=kap, a=a, b=1.0 / 30.0, cK=cK, mu1=mu1, mu3=mu3, e1=e1, e2=e2, ikh=ikh)


def d2(U: np.ndarray, axis: int, lo: str, hi: str) -> np.ndarray:
    """h^2 delta^2 along one array axis.

    Outside the unknown range the neighbour is the boundary value 0 on a
    Dirichlet face, or the mirror value U_{+1} of a Neumann face.
    """
    V = np.moveaxis(U, axis, 0)
    out = -2.0 * V
    out[1:] += V[:-1]
    out[:-1] += V[1:]
    if V.shape[0] > 1:
        if lo == "N":
            out[0] += V[1]
        if hi == "N":
            out[-1] += V[-2]
    return np.moveaxis(out, 0, axis)


class InPlane:
    """In-plane operators acting on (..., n'_y, n'_x) arrays with the x/y face rules."""

    def __init__(self, prob: Problem):
        self.bx = prob.axis_bc(0)
        self.by = prob.axis_bc(1)

    def Dx(self, U):
        return d2(U, U.ndim - 1, *self.bx)

    def Dy(self, U):
        return d2(U, U.ndim - 2, *self.by)

    def combo(self, U, c_id, c_lap, c_xy):
        """c_id U + c_lap (D_x + D_y) U + c_xy D_x D_y U."""
        dx = self.Dx(U)
        return c_id * U + c_lap * (dx + self.Dy(U)) + c_xy * self.Dy(dx)


def sommerfeld_QR(c: dict):
    """Coefficients (identity, D_x + D_y, D_x D_y) of Q and R in (3DDISCS).

    With D = h^2 delta^2:
      Q = e^{2ikh} mu3 [ (mu1 + (2ikh/3)(1/60 - mu1)) (D_x + D_y)
                         + 1/(30 mu3) D_x D_y + (1 - 2ikh/3 - 4 i (kh)^3 / 45) I ]
      R = e^{ikh} mu3 [ (4ikh/3)(1 + 2 kappa/15) I - (4ikh/3)(1/60 - mu1)(D_x + D_y) ]
    """
    ikh, mu1, mu3, kap = c["ikh"], c["mu1"], c["mu3"], c["kappa"]
    kh3 = (ikh / 1j) ** 3
    q = c["e2"] * mu3
    Q = (q * (1.0 - 2.0 * ikh / 3.0 - 4j * kh3 / 45.0),
         q * (mu1 + (2.0 * ikh / 3.0) * (1.0 / 60.0 - mu1)),
         q / (30.0 * mu3))
    r = c["e1"] * mu3
    R = (r * (4.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0),
         -r * (4.0 * ikh / 3.0) * (1.0 / 60.0 - mu1),
         0.0)
    return Q, R


def apply_A(prob: Problem, U: np.ndarray) -> np.ndarray:
    """y = A U, the h^2-scaled sixth-order compact operator with its closures."""
    U = np.asarray(U, dtype=np.complex128).reshape(prob.shape)
    c = coefficients(prob)
    ip = InPlane(prob)
    GU = ip.combo(U, 1.0, c["a"], c["b"])
    PU = ip.combo(U, c["kappa"] * c["cK"], 1.0, c["a"])
    AU = PU - 2.0 * GU
    AU[1:] += GU[:-1]
    AU[:-1] += GU[1:]
    lo, hi = prob.axis_bc(2)
    Q, R = sommerfeld_QR(c)
    if lo == "N":
        AU[0] += GU[1]
    elif lo == "S":
        AU[0] += ip.combo(U[1], *Q) + ip.combo(U[0], *R)
    if hi == "N":
        AU[-1] += GU[-2]
    elif hi == "S":
        AU[-1] += ip.combo(U[-2], *Q) + ip.combo(U[-1], *R)
    return AU


def apply_G_plane(prob: Problem, plane: np.ndarray) -> np.ndarray:
    """G applied to one z-plane (used for nonhomogeneous Dirichlet data)."""
    c = coefficients(prob)
    return InPlane(prob).combo(plane, 1.0, c["a"], c["b"])


def dirichlet_eigenvalue(prob: Problem, i: int, j: int, l: int) -> complex:
    """Closed-form eigenvalue of A for the Dirichlet sine mode (i, j, l).

    Section 3.4 (3DEGV): with s_r = sin^2(r pi h / 2),
      lambda = -4(s_i + s_j + s_l) + h^2k^2 + (8/3)(1 + h^2k^2/30)(s_i s_j + s_i s_l + s_j s_l)
               - (32/15) s_i s_j s_l - h^4k^4/12 + h^6k^6/360.
    Valid for the unit cube with all-Dirichlet faces.
    """
    h, kap = prob.h, prob.kappa
    s = [np.sin(r * np.pi * h / 2.0) ** 2 for r in (i, j, l)]
    return (-4.0 * sum(s) + kap
            + (8.0 / 3.0) * (1.0 + kap / 30.0) * (s[0] * s[1] + s[0] * s[2] + s[1] * s[2])
            - (32.0 / 15.0) * s[0] * s[1] * s[2] - kap ** 2 / 12.0 + kap ** 3 / 360.0)


def dirichlet_eigenvalue_p(prob: Problem, i: int, j: int, l: int) -> complex:
    """Closed-form eigenvalue of the 7-point A_p for the Dirichlet mode (i, j, l) (Section 3.4)."""
    h = prob.h
    s = [np.sin(r * np.pi * h / 2.0) ** 2 for r in (i, j, l)]
    return -4.0 * sum(s) + prob.kappa


def dirichlet_preconditioned_bounds(prob: Problem):
    """(min, max) over all Dirichlet sine modes of lambda / lambda^p, the
    eigenvalues 1 + d of A A_p^{-1} (eq. (3DEGV)) for real k and all-Dirichlet
    faces.  Evaluated for every mode (i, j, l) of the grid.  On a box with n_a
    unknowns per axis the sine modes have s_r = sin^2(r pi / (2 (n_a + 1)))
    (= sin^2(r pi h / 2) on the unit cube of eq. (3DEGV))."""
    if any(f != "D" for f in prob.bc) or complex(prob.k).imag != 0.0:
        raise ValueError("the closed-form spectrum needs real k and Dirichlet faces")
    kap = float(np.real(prob.kappa))
    s = [np.sin(np.arange(1, n + 1) * np.pi / (2.0 * (n + 1))) ** 2 for n in prob.n]
    si, sj, sl = np.meshgrid(s[0], s[1], s[2], indexing="ij", sparse=True)
    lp = -4.0 * (si + sj + sl) + kap
    lam = (lp + (8.0 / 3.0) * (1.0 + kap / 30.0) * (si * sj + si * sl + sj * sl)
           - (32.0 / 15.0) * si * sj * sl - kap ** 2 / 12.0 + kap ** 3 / 360.0)
    ratio = lam / lp
    return float(ratio.min()), float(ratio.max())
