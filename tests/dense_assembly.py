"""Independent row-by-row assembly of A and A_p as dense matrices (n <= 8).

Second definition of the operators, used only by tests.  Each row is built
from the 27 neighbour weights of eq. (scheme) (left-hand side times h^2),
then every neighbour that is not an unknown is substituted explicitly:

* Dirichlet boundary node -> 0 (homogeneous data);
* x/y ghost node on a Neumann face -> its mirror node (U_{-1} = U_1);
* z ghost node on a Neumann face -> its mirror node (eq. (3DN), beta = 0);
* z ghost plane on a Sommerfeld face -> the weights that multiply the ghost
  plane form exactly the in-plane operator on the left of eq. (3DDISCS), so
  that sum is replaced by the 9-point stencils of its right-hand side acting
  on the first interior plane and on the boundary plane.

The Sommerfeld stencil coefficients are written out here again from
(3DDISCS), not imported from the oracle.
"""
from __future__ import annotations

import cmath
import itertools

import numpy as np

from oracle.grid import Problem


def _c1(d):
    return -2.0 if d == 0 else 1.0


def scheme_weight(d, kap):
    """Weight of neighbour offset d = (dx, dy, dz) in h^2 * LHS of (scheme)."""
    dx, dy, dz = d
    a = (1.0 + kap / 30.0) / 6.0
    cK = 1.0 - kap / 12.0 + kap * kap / 360.0
    w = 0.0
    if dy == 0 and dz == 0:
        w += _c1(dx)
    if dx == 0 and dz == 0:
        w += _c1(dy)
    if dx == 0 and dy == 0:
        w += _c1(dz)
    if dz == 0:
        w += a * _c1(dx) * _c1(dy)
    if dy == 0:
        w += a * _c1(dx) * _c1(dz)
    if dx == 0:
        w += a * _c1(dy) * _c1(dz)
    w += _c1(dx) * _c1(dy) * _c1(dz) / 30.0
    if d == (0, 0, 0):
        w += kap * cK
    return w


def _sommerfeld_stencils(prob: Problem):
    """9-point (dx, dy) -> weight maps of Q and R in (3DDISCS)."""
    k, h = prob.k, prob.h
    kap = (k * h) ** 2
    ikh = 1j * k * h
    mu3 = 1.0 / (1.0 + (2.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0))
    mu1 = (ikh / 90.0 + (1.0 + kap / 30.0) / (6.0 * mu3)) / (1.0 + 2.0 * ikh / 3.0)
    e1, e2 = cmath.exp(ikh), cmath.exp(2.0 * ikh)
    lap_coef_Q = mu1 + (2.0 * ikh / 3.0) * (1.0 / 60.0 - mu1)
    id_Q = 1.0 - 2.0 * ikh / 3.0 - 4j * (k * h) ** 3 / 45.0
    Q, R = {}, {}
    for dx, dy in itertools.product((-1, 0, 1), repeat=2):
        lap = (_c1(dx) if dy == 0 else 0.0) + (_c1(dy) if dx == 0 else 0.0)
        xy = _c1(dx) * _c1(dy)
        ident = 1.0 if (dx, dy) == (0, 0) else 0.0
        Q[(dx, dy)] = e2 * mu3 * (lap_coef_Q * lap + xy / (30.0 * mu3) + id_Q * ident)
        R[(dx, dy)] = e1 * mu3 * ((4.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0) * ident
                                  - (4.0 * ikh / 3.0) * (1.0 / 60.0 - mu1) * lap)
    return Q, R


class _Index:
    def __init__(self, prob: Problem):
        self.prob = prob
        self.rng = [prob.q_range(a) for a in range(3)]
        self.dims = prob.dims
        self.nz = prob.n[2]

    def lin(self, q):
        ix, iy, iz = (q[a] - self.rng[a][0] for a in range(3))
        nx, ny, _ = self.dims
        return ix + nx * (iy + ny * iz)

    def resolve_xy(self, q):
        """Map a node whose x/y index may be off-range to [(weight, q')] (z untouched)."""
        q = list(q)
        for a in (0, 1):
            lo, hi = self.rng[a]
            code_lo, code_hi = self.prob.axis_bc(a)
            n = self.prob.n[a]
            if q[a] < lo:
                if code_lo == "D" and q[a] == 0:
                    return []
                if code_lo == "N" and q[a] == -1:
                    q[a] = 1
                else:
                    raise AssertionError("unexpected x/y offset")
            elif q[a] > hi:
                if code_hi == "D" and q[a] == n + 1:
                    return []
                if code_hi == "N" and q[a] == n + 2:
                    q[a] = n
                else:
                    raise AssertionError("unexpected x/y offset")
        return [(1.0, tuple(q))]


def dense_A(prob: Problem) -> np.ndarray:
    idx = _Index(prob)
    N = int(np.prod(prob.dims))
    A = np.zeros((N, N), dtype=np.complex128)
    kap = prob.kappa
    Q, R = _sommerfeld_stencils(prob)
    zlo, zhi = idx.rng[2]
    blo, bhi = prob.axis_bc(2)
    nz = prob.n[2]
    for q in itertools.product(*[range(a, b + 1) for a, b in idx.rng]):
        row = idx.lin(q)

        def add(weight, node):
            for w2, q2 in idx.resolve_xy(node):
                A[row, idx.lin(q2)] += weight * w2

        for d in itertools.product((-1, 0, 1), repeat=3):
            w = scheme_weight(d, kap)
            node = (q[0] + d[0], q[1] + d[1], q[2] + d[2])
            qz = node[2]
            if zlo <= qz <= zhi:
                add(w, node)
            elif qz == 0 and blo == "D" or qz == nz + 1 and bhi == "D":
                continue                                   # boundary value 0
            elif qz == -1 and blo == "N":
                add(w, (node[0], node[1], 1))              # mirror
            elif qz == nz + 2 and bhi == "N":
                add(w, (node[0], node[1], nz))
            elif qz in (-1, nz + 2):
                continue                                   # Sommerfeld: replaced below
            else:
                raise AssertionError("unexpected z offset")
        if q[2] == 0 and blo == "S":
            for (dx, dy), w in Q.items():
                add(w, (q[0] + dx, q[1] + dy, 1))
            for (dx, dy), w in R.items():
                add(w, (q[0] + dx, q[1] + dy, 0))
        if q[2] == nz + 1 and bhi == "S":
            for (dx, dy), w in Q.items():
                add(w, (q[0] + dx, q[1] + dy, nz))
            for (dx, dy), w in R.items():
                add(w, (q[0] + dx, q[1] + dy, nz + 1))
    return A


def dense_Ap(prob: Problem) -> np.ndarray:
    """7-point second-order operator of (3DAP), assembled row by row."""
    idx = _Index(prob)
    N = int(np.prod(prob.dims))
    A = np.zeros((N, N), dtype=np.complex128)
    zlo, zhi = idx.rng[2]
    blo, bhi = prob.axis_bc(2)
    nz = prob.n[2]
    alpha = 2j * prob.k * prob.h
    for q in itertools.product(*[range(a, b + 1) for a, b in idx.rng]):
        row = idx.lin(q)

        def add(weight, node):
            for w2, q2 in idx.resolve_xy(node):
                A[row, idx.lin(q2)] += weight * w2

        add(-6.0 + prob.kappa, q)
        for a in range(3):
            for s in (-1, 1):
                node = list(q)
                node[a] += s
                node = tuple(node)
                qz = node[2]
                if a < 2 or zlo <= qz <= zhi:
                    add(1.0, node)
                elif qz == 0 and blo == "D" or qz == nz + 1 and bhi == "D":
                    continue
                elif qz == -1:                  # U_{-1} = U_1 (+ 2ikh U_0 for S)
                    add(1.0, (q[0], q[1], 1))
                    if blo == "S":
                        add(alpha, (q[0], q[1], 0))
                elif qz == nz + 2:
                    add(1.0, (q[0], q[1], nz))
                    if bhi == "S":
                        add(alpha, (q[0], q[1], nz + 1))
    return A
