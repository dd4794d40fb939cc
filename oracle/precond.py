"""The second-order 7-point preconditioner A_p and its direct inverse.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.

Section 3.3, eq. (3DAP), h^2-scaled:

  A_p = A^0_{beta_x} (x) I (x) I + I (x) A^0_{beta_y} (x) I + I (x) I (x) A_{alpha_z, beta_z},

i.e. A_p = D_x + D_y + T_z + kappa I with kappa = (kh)^2, where

* D_x, D_y are the 3-point second differences of the scheme (zero ghost on a
  Dirichlet pair, beta = 0; mirror ghost on a Neumann pair, beta = 1, which
  puts 1 + beta = 2 in the corner entries of Lambda^beta);
* T_z = tridiag(1, -2, 1) with 2 in the corner entry next to a Neumann or
  Sommerfeld z face (beta_z = 1) and an extra alpha_z = 2 i k h on the
  diagonal entry of a Sommerfeld face (second-order central closure of
  u_z + i k u = 0).  The two z faces are treated independently.

Inverse by separation of variables (Section 3.3: FFT-type transforms in x
and y, one tridiagonal solve per transverse mode in z).  With M = n + 1:

* Dirichlet pair (n unknowns): W_qm = sin(pi q m / M), q, m = 1..n,
  W^{-1} = (2/M) W^T;
* Neumann pair (n + 2 unknowns): W_qm = cos(pi q m / M), q, m = 0..M,
  W^{-1} = (2/M) C W^T C with C = diag(1/2, 1, ..., 1, 1/2);
* in both cases the eigenvalue of mode m is lambda(m) = -4 sin^2(pi m / (2M)).

The transforms are evaluated with scipy's type-1 DST/DCT (plain library
primitives).  Each mode (m_x, m_y) then solves
(T_z + (kappa + lambda_x + lambda_y) I) zhat = rhat by Gaussian elimination
without pivoting (the Thomas algorithm).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .grid import Problem
from .scheme import d2


class SingularPreconditioner(ArithmeticError):
    """A zero or non-finite pivot in a z tridiagonal solve (k^2 on the 7-point spectrum)."""


PIVOT_RTOL = 1e-12


def apply_Ap(prob: Problem, U: np.ndarray) -> np.ndarray:
    """y = A_p U with a 7-point stencil (independent of the inverse below)."""
    U = np.asarray(U, dtype=np.complex128).reshape(prob.shape)
    bx, by = prob.axis_bc(0), prob.axis_bc(1)
    out = d2(U, 2, *bx) + d2(U, 1, *by) + prob.kappa * U
    # z: second difference with the ghost rules of the z faces
    Tz = -2.0 * U
    Tz[1:] += U[:-1]
    Tz[:-1] += U[1:]
    lo, hi = prob.axis_bc(2)
    alpha = 2j * prob.k * prob.h
    if lo in "NS":
        Tz[0] += U[1]
        if lo == "S":
            Tz[0] += alpha * U[0]
    if hi in "NS":
        Tz[-1] += U[-2]
        if hi == "S":
            Tz[-1] += alpha * U[-1]
    return out + Tz


def mode_eigenvalues(prob: Problem, ax: int) -> np.ndarray:
    n = prob.n[ax]
    M = n + 1
    lo, _ = prob.axis_bc(ax)
    m = np.arange(1, n + 1) if lo == "D" else np.arange(0, M + 1)
    return -4.0 * np.sin(np.pi * m / (2.0 * M)) ** 2


def _end_weights(length: int) -> np.ndarray:
    w = np.ones(length)
    w[0] = w[-1] = 0.5
    return w


def forward_transform(R: np.ndarray, axis: int, code: str) -> np.ndarray:
    """c = W^{-1} r along one array axis ('D': sine, 'N': cosine basis)."""
    L = R.shape[axis]
    if code == "D":
        M = L + 1
        return sfft.dst(R, type=1, axis=axis) / M
    M = L - 1
    w = _end_weights(L).reshape([-1 if a == axis else 1 for a in range(R.ndim)])
    return w * sfft.dct(R, type=1, axis=axis) / M


def inverse_transform(C: np.ndarray, axis: int, code: str) -> np.ndarray:
    """r = W c along one array axis."""
    L = C.shape[axis]
    if code == "D":
        return 0.5 * sfft.dst(C, type=1, axis=axis)
    w = _end_weights(L).reshape([-1 if a == axis else 1 for a in range(C.ndim)])
    return 0.5 * sfft.dct(C / w, type=1, axis=axis)


def z_tridiagonal(prob: Problem):
    """(sub, diag, sup) of T_z as arrays over the n'_z rows (sub[0], sup[-1] unused)."""
    nz = prob.shape[0]
    sub = np.ones(nz, dtype=np.complex128)
    sup = np.ones(nz, dtype=np.complex128)
    diag = np.full(nz, -2.0, dtype=np.complex128)
    lo, hi = prob.axis_bc(2)
    alpha = 2j * prob.k * prob.h
    if lo in "NS":
        sup[0] = 2.0
        if lo == "S":
            diag[0] += alpha
    if hi in "NS":
        sub[-1] = 2.0
        if hi == "S":
            diag[-1] += alpha
    return sub, diag, sup


def thomas(sub, diag, sup, shift: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Solve (T + diag(shift)) X = R along axis 0 for every transverse mode.

    shift has the transverse shape (n'_y, n'_x); R has shape (n'_z, n'_y, n'_x).
    Gaussian elimination without pivoting; a pivot smaller than
    PIVOT_RTOL * (4 + |shift|) or non-finite raises SingularPreconditioner.
    """
    nz = R.shape[0]
    scale = 4.0 + np.abs(shift)
    cp = np.zeros(R.shape, dtype=np.complex128)
    dp = np.zeros(R.shape, dtype=np.complex128)
    prev_c = None
    for i in range(nz):
        piv = diag[i] + shift
        if i > 0:
            piv = piv - sub[i] * prev_c
        if not np.all(np.isfinite(piv)) or np.any(np.abs(piv) <= PIVOT_RTOL * scale):
            raise SingularPreconditioner(f"zero pivot in z row {i}")
        cp[i] = sup[i] / piv
        dp[i] = (R[i] - (sub[i] * dp[i - 1] if i > 0 else 0.0)) / piv
        prev_c = cp[i]
    X = np.empty_like(R)
    X[-1] = dp[-1]
    for i in range(nz - 2, -1, -1):
        X[i] = dp[i] - cp[i] * X[i + 1]
    return X


def apply_Pinv(prob: Problem, R: np.ndarray) -> np.ndarray:
    """z = A_p^{-1} r by x/y transforms and per-mode z tridiagonal solves."""
    R = np.asarray(R, dtype=np.complex128).reshape(prob.shape)
    bx, by = prob.axis_bc(0)[0], prob.axis_bc(1)[0]
    C = forward_transform(R, 2, bx)
    C = forward_transform(C, 1, by)
    lx = mode_eigenvalues(prob, 0)
    ly = mode_eigenvalues(prob, 1)
    shift = prob.kappa + ly[:, None] + lx[None, :]
    sub, diag, sup = z_tridiagonal(prob)
    Z = thomas(sub, diag, sup, shift, C)
    Z = inverse_transform(Z, 1, by)
    return inverse_transform(Z, 2, bx)
