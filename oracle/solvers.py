"""Krylov solvers of the oracle: right-preconditioned GMRES(m), flexible
GMRES(m) and the SKS two-level iteration.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.

* Right preconditioning (Section 2, eq. (AAP)): solve A A_p^{-1} Y = F, then
  A_p U = Y.  GMRES(m) builds an Arnoldi basis of A A_p^{-1} with modified
  Gram-Schmidt, updates a QR factorisation of the Hessenberg matrix with
  complex Givens rotations, and restarts after m steps.  The test on the true
  residual ||F - A U||_2 / ||F||_2 <= tol (Section 4.1) is made at the end of
  each cycle; inside a cycle the least-squares residual serves as estimate.
* Flexible GMRES stores the preconditioned vectors z_j = M_j^{-1} v_j, so the
  preconditioner may change (or be inexact) from step to step.
* Chebyshev acceleration (Section 2, Theorem 2 and its citation; Section 4):
  the classical Chebyshev iteration for a real spectrum [alpha, beta],
  0 < alpha, applied to the right-preconditioned system A A_p^{-1} Y = F and
  written for U = A_p^{-1} Y; the paper takes alpha, beta from the exact
  eigenvalues (3DEGV) of the Dirichlet problem.
* SKS (Section 2, Algorithm 1): Y = F; repeat U = A_p^{-1} Y, r = F - A U,
  eps = ||r|| / ||F||, stop if eps <= tol, Y = Y + r.  The loop condition of
  the printed algorithm is read as "while j <= maxit and eps > tol", with
  eps = infinity on entry; divergence ("div" in Tables 4, 6, 8) is flagged
  when eps exceeds 1e4 or is not finite.

All iteration counts are numbers of A A_p^{-1} applications, as in the
paper's tables.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    iters: int = 0
    rel_resid: float = np.inf
    status: str = "not_converged"     # 'ok', 'not_converged', 'diverged'
    history: list = field(default_factory=list)


def _norm(v):
    return float(np.sqrt(np.vdot(v, v).real))


def givens(a: complex, b: float):
    """Complex rotation (c real, s complex) with [c s; -conj(s) c][a; b] = [r; 0]."""
    if b == 0.0:
        return 1.0, 0.0j, a
    if a == 0.0:
        return 0.0, 1.0 + 0.0j, complex(b)
    t = np.hypot(abs(a), b)
    ph = a / abs(a)
    return abs(a) / t, ph * np.conj(b) / t, ph * t


def gmres(A, Pinv, F, x0=None, restart=30, tol=1e-10, maxit=1000, flexible=False):
    """Right-preconditioned restarted GMRES; A and Pinv are callables on arrays.

    With flexible=True the preconditioned basis Z is stored and the update is
    U += Z y (FGMRES); otherwise U += Pinv(V y).
    """
    shape = F.shape
    F = F.reshape(-1)
    U = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.complex128).reshape(-1)
    normF = _norm(F)
    info = SolveInfo()
    if normF == 0.0:
        info.status, info.rel_resid = "ok", 0.0
        return np.zeros(shape, dtype=np.complex128), info
    r = F - A(U.reshape(shape)).reshape(-1)
    beta = _norm(r)
    info.rel_resid = beta / normF
    while True:
        if beta <= tol * normF:
            info.status = "ok"
            break
        if info.iters >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, F.size), dtype=np.complex128)
        Z = np.zeros((m, F.size), dtype=np.complex128) if flexible else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            z = Pinv(V[j].reshape(shape)).reshape(-1)
            if flexible:
                Z[j] = z
            w = A(z.reshape(shape)).reshape(-1)
            info.iters += 1
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):              # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            c, s, rr = givens(H[j, j], H[j + 1, j].real)
            cs[j], sn[j] = c, s
            H[j, j], H[j + 1, j] = rr, 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            j_done = j + 1
            est = abs(g[j + 1]) / normF
            info.history.append(est)
            if est <= tol or info.iters >= maxit:
                break
        # least-squares solution of the triangular system
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        if flexible:
            U = U + y @ Z[:j_done]
        else:
            U = U + Pinv((y @ V[:j_done]).reshape(shape)).reshape(-1)
        r = F - A(U.reshape(shape)).reshape(-1)
        beta = _norm(r)
        info.rel_resid = beta / normF
    return U.reshape(shape), info


def sks(A, Pinv, F, tol=1e-10, maxit=100, diverge=1e4):
    """Algorithm 1 (SKS) with zero initial guess."""
    normF = _norm(F.reshape(-1))
    info = SolveInfo()
    Y = F.copy()
    U = np.zeros_like(F)
    if normF == 0.0:
        info.status, info.rel_resid = "ok", 0.0
        return U, info
    for _ in range(maxit):
        U = Pinv(Y)
        r = F - A(U)
        eps = _norm(r.reshape(-1)) / normF
        info.iters += 1
        info.history.append(eps)
        info.rel_resid = eps
        if eps <= tol:
            info.status = "ok"
            return U, info
        if not np.isfinite(eps) or eps > diverge:
            info.status = "diverged"
            return U, info
        Y = Y + r
    return U, info


def sks_correction(A, Pinv, F, x0=None, tol=1e-10, maxit=100, diverge=1e4):
    """SKS in correction form: U += Pinv(r), r = F - A U.

    With x0 = 0 its iterates equal Algorithm 1's in exact arithmetic
    (U_{j+1} = Pinv(Y_j + r_j) = U_j + Pinv(r_j)); it is the form used when
    the preconditioner is inexact (lower precision).
    """
    normF = _norm(F.reshape(-1))
    info = SolveInfo()
    U = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.complex128)
    if normF == 0.0:
        info.status, info.rel_resid = "ok", 0.0
        return np.zeros_like(F), info
    r = F - A(U)
    for _ in range(maxit):
        U = U + Pinv(r)
        r = F - A(U)
        eps = _norm(r.reshape(-1)) / normF
        info.iters += 1
        info.history.append(eps)
        info.rel_resid = eps
        if eps <= tol:
            info.status = "ok"
            return U, info
        if not np.isfinite(eps) or eps > diverge:
            info.status = "diverged"
            return U, info
    return U, info


def chebyshev(A, Pinv, F, alpha: float, beta: float, tol=1e-10, maxit=100, diverge=1e4):
    """Chebyshev acceleration on A A_p^{-1} Y = F, spectrum in [alpha, beta].

    With theta = (alpha + beta) / 2, delta = (beta - alpha) / 2 and
    sigma = theta / delta, the textbook recurrence in Y reads
      d_0 = r_0 / theta,  rho_0 = 1 / sigma,
      Y_{k+1} = Y_k + d_k,  r_{k+1} = r_k - A A_p^{-1} d_k,
      rho_{k+1} = 1 / (2 sigma - rho_k),
      d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) r_{k+1};
    with e_k = A_p^{-1} d_k it becomes, for U = A_p^{-1} Y,
      U_{k+1} = U_k + e_k,  e_{k+1} = rho_{k+1} rho_k e_k + (2 rho_{k+1} / delta) A_p^{-1} r_{k+1}.
    The residual r = F - A U is recomputed every iteration.  Zero initial
    guess; iterations are counted as A A_p^{-1} applications."""
    if not (0.0 < alpha < beta):
        raise ValueError("Chebyshev acceleration needs 0 < alpha < beta")
    theta, delta = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    sigma = theta / delta
    normF = _norm(F.reshape(-1))
    info = SolveInfo()
    U = np.zeros_like(F)
    if normF == 0.0:
        info.status, info.rel_resid = "ok", 0.0
        return U, info
    r = F.copy()
    rho = 1.0 / sigma
    e = Pinv(r) / theta
    for _ in range(maxit):
        U = U + e
        r = F - A(U)
        eps = _norm(r.reshape(-1)) / normF
        info.iters += 1
        info.history.append(eps)
        info.rel_resid = eps
        if eps <= tol:
            info.status = "ok"
            return U, info
        if not np.isfinite(eps) or eps > diverge:
            info.status = "diverged"
            return U, info
        rho_next = 1.0 / (2.0 * sigma - rho)
        e = rho_next * rho * e + (2.0 * rho_next / delta) * Pinv(r)
        rho = rho_next
    return U, info


def psi_order(eps_h: float, eps_gh: float, gamma: float) -> float:
    """Order estimate psi of eq. (PSI): (ln eps^{gamma h} - ln eps^h) / ln gamma,
    with eps^h = ||r_2|| / ||r_1|| from the first two SKS iterations on grid h."""
    return (np.log(eps_gh) - np.log(eps_h)) / np.log(gamma)
