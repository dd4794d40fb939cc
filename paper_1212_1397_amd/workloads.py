"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and names grid sizes; it holds none of
the method's arithmetic (no operator, right-hand side or solver code), so both
the CPU oracle's callers and the GPU path can take their inputs from it.

Workloads (unit cube, n interior nodes per axis, h = 1/(n+1)):
  * ``dirichlet-32``: 32^3, all faces Dirichlet, k = 10, manufactured
    u = sin(pi x) sin(2 pi y) sin(3 pi z)  (GMRES(20), tol 1e-10);
  * ``dns-128``: 128^3 interior nodes, x Dirichlet / y Neumann / z Sommerfeld
    faces (128 x 130 x 130 unknowns), k = 40 + 0.4i, one Gaussian source of
    width sigma = 4h and amplitude 1 at a seeded centre in [0.25, 0.75]^3;
  * ``dns-256``: 256^3 interior nodes, same faces (256 x 258 x 258 unknowns),
    k = 80 + 0.8i, eight Gaussian sources of width 4h with amplitudes drawn
    from N(0,1) + i N(0,1) at seeded centres in [0.25, 0.75]^3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    k: complex
    bc: str
    nsrc: int            # 0: manufactured sine source (dirichlet-32)
    seed: int
    complex_amps: bool
    restart: int
    tol: float

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def sigma(self) -> float:
        return 4.0 * self.h


WORKLOADS = {
    "dirichlet-32": Workload("dirichlet-32", 32, 10.0 + 0j, "DDDDDD", 0, 1, False, 20, 1e-10),
    "dns-128": Workload("dns-128", 128, 40.0 + 0.4j, "DDNNSS", 1, 2, False, 30, 1e-8),
    "dns-256": Workload("dns-256", 256, 80.0 + 0.8j, "DDNNSS", 8, 3, True, 30, 1e-8),
}


def gaussian_sources(w: Workload):
    """(centres (nsrc, 3), amplitudes (nsrc,) complex, sigma) drawn from the seed."""
    rng = np.random.default_rng(w.seed)
    centres = rng.uniform(0.25, 0.75, size=(w.nsrc, 3))
    if w.complex_amps:
        amps = rng.standard_normal(w.nsrc) + 1j * rng.standard_normal(w.nsrc)
    else:
        amps = np.ones(w.nsrc, dtype=np.complex128)
    return centres, amps.astype(np.complex128), w.sigma


def random_field(shape, seed: int) -> np.ndarray:
    """Complex128 array with N(0,1) + i N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_sources(nsrc: int, seed: int, h: float, lo: float = 0.25, hi: float = 0.75):
    """Gaussian sources (width 4h) at seeded centres with complex normal amplitudes."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(nsrc, 3))
    amps = rng.standard_normal(nsrc) + 1j * rng.standard_normal(nsrc)
    return centres, amps, 4.0 * h


def init_net_params(layers, seed: int):
    """He-normal initial weights of the correction network: for each
    (name, Cin, Cout) in `layers`, W ~ N(0, 2 / (27 Cin)) of shape
    (Cout, Cin, 3, 3, 3) and b = 0; the last layer's weights are scaled by
    1e-2 so that the initial correction is small.  Returns {name: (W, b)}."""
    rng = np.random.default_rng(seed)
    out = {}
    for i, (name, cin, cout) in enumerate(layers):
        W = rng.standard_normal((cout, cin, 3, 3, 3)) * np.sqrt(2.0 / (27 * cin))
        if i == len(layers) - 1:
            W *= 1e-2
        out[name] = (W, np.zeros(cout))
    return out


@dataclass(frozen=True)
class BatchInstance:
    n: int
    k: complex
    bc: str
    centres: np.ndarray
    amps: np.ndarray
    sigma: float

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)


def batch_workload(count: int = 96, seed: int = 4, sizes=(48, 64, 96, 128, 160)):
    """The many-solve workload: `count` independent problems with n drawn
    uniformly from `sizes`, k = kr (1 + 0.01 i) with kr ~ U[10, 60], faces
    all Dirichlet or x Dirichlet / y Neumann / z Sommerfeld (equally likely),
    one Gaussian source of width 4h and amplitude 1 at a seeded centre in
    [0.25, 0.75]^3."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        kr = float(rng.uniform(10.0, 60.0))
        bc = "DDDDDD" if rng.integers(2) == 0 else "DDNNSS"
        centre = rng.uniform(0.25, 0.75, size=(1, 3))
        h = 1.0 / (n + 1)
        out.append(BatchInstance(n, kr * (1 + 0.01j), bc, centre, np.ones(1, dtype=np.complex128), 4.0 * h))
    return out
