"""FP64 CPU oracle for the sixth-order compact Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference against which the HIP implementation is checked.  It
shares no code with the GPU library and must only be imported by the test
suite, the smoke check and the CPU-baseline leg of the benchmark.

Contents (each module cites the passages of the paper it follows):
  grid      - problem, faces and unknown layout (Section 1, Section 3.3, Section 4.2)
  functions - analytic separable sources with exact derivatives
  scheme    - the 27-point compact operator A with its closures (Section 3.1-3.2)
  rhs       - the compact right-hand side F with face terms (Section 3.1-3.2)
  precond   - the 7-point preconditioner A_p and its direct inverse (Section 3.3)
  solvers   - GMRES(m), flexible GMRES(m), SKS (Section 2, Algorithm 1),
              Chebyshev acceleration (Section 2, Theorem 2)
  onedim    - the 1D model problem (Section 2, Table 2)
"""
from .grid import Problem, UnsupportedBC, FACES
from .scheme import (apply_A, coefficients, dirichlet_eigenvalue, dirichlet_eigenvalue_p,
                     dirichlet_preconditioned_bounds)
from .precond import apply_Ap, apply_Pinv, SingularPreconditioner
from .rhs import rhs
from .solvers import gmres, sks, sks_correction, chebyshev, psi_order, SolveInfo
from . import functions


def solve(prob: Problem, F, method="gmres", restart=30, tol=1e-10, maxit=1000, x0=None):
    """Solve A U = F with the preconditioner A_p (method: gmres, fgmres, sks, sks_correction,
    chebyshev; the last uses the closed-form Dirichlet spectrum of A A_p^{-1})."""
    A = lambda U: apply_A(prob, U)
    P = lambda R: apply_Pinv(prob, R)
    if method in ("gmres", "fgmres"):
        return gmres(A, P, F, x0=x0, restart=restart, tol=tol, maxit=maxit,
                     flexible=(method == "fgmres"))
    if method == "sks":
        return sks(A, P, F, tol=tol, maxit=maxit)
    if method == "sks_correction":
        return sks_correction(A, P, F, x0=x0, tol=tol, maxit=maxit)
    if method == "chebyshev":
        lo, hi = dirichlet_preconditioned_bounds(prob)
        return chebyshev(A, P, F, lo, hi, tol=tol, maxit=maxit)
    raise ValueError(method)
