"""Grid and boundary-condition model of the oracle.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.

Domain and faces follow Section 1, eqs. (problem) and (bc): the box
[0, (nx+1)h] x [0, (ny+1)h] x [0, (nz+1)h] with one boundary condition per
face, Dirichlet 'D' (u = 0), Neumann 'N' (u_n = 0) or Sommerfeld-like 'S'
(u_n - i k u = 0, i.e. u_z + i k u = 0 at z = 0 and u_z - i k u = 0 at the top).

Grid (Section 3.3 and Section 4.2): nodes q*h, q = 0..n+1 on every axis with
a common step h (the paper's h = 1/(N+1) on the unit cube).  Dirichlet faces
carry no unknowns; a Neumann or Sommerfeld face makes its boundary plane an
unknown plane (the paper's N_z = N+1 for one Neumann face, N_z = N+2 for two
Sommerfeld faces).  Unknown vectors are stored as complex arrays of shape
(n'_z, n'_y, n'_x), x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FACES = ("x-", "x+", "y-", "y+", "z-", "z+")


class UnsupportedBC(ValueError):
    """Face combination for which the paper gives no preconditioner (Section 3.3)."""


@dataclass(frozen=True)
class Problem:
    n: tuple          # interior node counts (nx, ny, nz)
    h: float          # grid step, the same on every axis
    k: complex        # wavenumber (complex allowed)
    bc: tuple         # six face codes in FACES order

    def __post_init__(self):
        if len(self.n) != 3 or min(self.n) < 1:
            raise ValueError("n must hold three counts >= 1")
        if not self.h > 0:
            raise ValueError("h must be positive")
        if len(self.bc) != 6 or any(b not in "DNS" for b in self.bc):
            raise ValueError("bc must be six codes from 'D', 'N', 'S'")
        for ax in (0, 1):
            lo, hi = self.bc[2 * ax], self.bc[2 * ax + 1]
            if "S" in (lo, hi):
                raise UnsupportedBC("Sommerfeld faces are supported on z only")
            if lo != hi:
                raise UnsupportedBC("x and y faces must be a D/D or N/N pair")

    @staticmethod
    def cube(n: int, k: complex, bc="DDDDDD") -> "Problem":
        """Unit cube with n interior nodes per axis, h = 1/(n+1)."""
        return Problem((n, n, n), 1.0 / (n + 1), complex(k), tuple(bc))

    @property
    def kappa(self) -> complex:
        """(k h)^2."""
        return (self.k * self.h) ** 2

    def axis_bc(self, ax: int):
        return self.bc[2 * ax], self.bc[2 * ax + 1]

    def q_range(self, ax: int):
        """First and last node index q holding an unknown on axis ax."""
        lo, hi = self.axis_bc(ax)
        n = self.n[ax]
        return (0 if lo != "D" else 1), (n + 1 if hi != "D" else n)

    @property
    def dims(self):
        """Unknown counts (n'_x, n'_y, n'_z)."""
        out = []
        for ax in range(3):
            a, b = self.q_range(ax)
            out.append(b - a + 1)
        return tuple(out)

    @property
    def shape(self):
        """Array shape (n'_z, n'_y, n'_x) of an unknown vector."""
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def coords(self, ax: int) -> np.ndarray:
        a, b = self.q_range(ax)
        return np.arange(a, b + 1) * self.h

    def points(self):
        return tuple(self.coords(ax) for ax in range(3))

    def length(self, ax: int) -> float:
        return (self.n[ax] + 1) * self.h

    def zeros(self):
        return np.zeros(self.shape, dtype=np.complex128)
