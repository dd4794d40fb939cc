"""Analytic one-dimensional factors with derivatives of any order, and
separable sums of their products.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.

The compact right-hand side of the sixth-order scheme (Section 3.1, eq.
(scheme)) and the boundary closures (eqs. (3DN), (3DIMP), (3DDISCS)) need
derivatives of the source f up to fourth order, including mixed ones.  Every
source used by the tests and benchmarks is a finite sum of separable products
f(x, y, z) = sum_s c_s X_s(x) Y_s(y) Z_s(z), so mixed derivatives factor into
products of one-dimensional derivatives, each available in closed form here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


class Factor:
    """A smooth complex function of one variable, differentiable to any order."""

    def d(self, x: np.ndarray, order: int) -> np.ndarray:  # pragma: no cover
        raise NotImplementedError

    def __call__(self, x):
        return self.d(np.asarray(x, dtype=np.float64), 0)

    def __mul__(self, other: "Factor") -> "Factor":
        return Product(self, other)

    def __add__(self, other: "Factor") -> "Factor":
        return Sum(self, other)


@dataclass
class Poly(Factor):
    """Polynomial with coefficients in increasing powers."""
    coeffs: tuple

    def d(self, x, order):
        p = np.polynomial.Polynomial(np.asarray(self.coeffs, dtype=np.complex128))
        return p.deriv(order)(x) if order else p(x)


@dataclass
class Exp(Factor):
    """exp(c x) for complex c; the n-th derivative is c**n exp(c x)."""
    c: complex

    def d(self, x, order):
        return (self.c ** order) * np.exp(self.c * x)


@dataclass
class Cos(Factor):
    """cos(w x + phi); the n-th derivative is w**n cos(w x + phi + n pi/2)."""
    w: float
    phi: float = 0.0

    def d(self, x, order):
        return (self.w ** order) * np.cos(self.w * x + self.phi + order * math.pi / 2) + 0j


def Sin(w: float) -> Cos:
    """sin(w x) = cos(w x - pi/2)."""
    return Cos(w, -math.pi / 2)


@dataclass
class Gauss(Factor):
    """exp(-(x-c)^2 / (2 s^2)).

    The n-th derivative is (-1/s)^n He_n((x-c)/s) exp(-(x-c)^2/(2 s^2)) with
    He_n the probabilists' Hermite polynomial (He_0 = 1, He_1 = t,
    He_{n+1} = t He_n - n He_{n-1}).
    """
    c: float
    s: float

    def d(self, x, order):
        t = (x - self.c) / self.s
        he_prev, he = np.ones_like(t), t
        if order == 0:
            he = he_prev
        else:
            for n in range(1, order):
                he_prev, he = he, t * he - n * he_prev
        return ((-1.0 / self.s) ** order) * he * np.exp(-0.5 * t * t) + 0j


@dataclass
class Product(Factor):
    """Product of two factors, differentiated with the Leibniz rule."""
    a: Factor
    b: Factor

    def d(self, x, order):
        out = np.zeros(np.shape(x), dtype=np.complex128)
        for j in range(order + 1):
            out = out + math.comb(order, j) * self.a.d(x, j) * self.b.d(x, order - j)
        return out


@dataclass
class Sum(Factor):
    """Sum of two factors."""
    a: Factor
    b: Factor

    def d(self, x, order):
        return self.a.d(x, order) + self.b.d(x, order)


@dataclass
class Term:
    """One separable product c * X(x) * Y(y) * Z(z)."""
    c: complex
    fx: Factor
    fy: Factor
    fz: Factor


class Separable:
    """f(x, y, z) = sum of separable Terms.

    ``deriv(pts, (ax, ay, az))`` evaluates the mixed derivative
    d^{ax+ay+az} f / dx^ax dy^ay dz^az on the tensor grid pts = (x, y, z),
    returning an array of shape (len(z), len(y), len(x)) (x fastest).
    """

    def __init__(self, terms):
        self.terms = list(terms)

    def __add__(self, other: "Separable") -> "Separable":
        return Separable(self.terms + other.terms)

    def scaled(self, s: complex) -> "Separable":
        return Separable([Term(t.c * s, t.fx, t.fy, t.fz) for t in self.terms])

    def deriv(self, pts, orders) -> np.ndarray:
        x, y, z = (np.asarray(p, dtype=np.float64) for p in pts)
        ax, ay, az = orders
        out = np.zeros((len(z), len(y), len(x)), dtype=np.complex128)
        for t in self.terms:
            X = t.fx.d(x, ax)
            Y = t.fy.d(y, ay)
            Z = t.fz.d(z, az)
            out += t.c * Z[:, None, None] * Y[None, :, None] * X[None, None, :]
        return out


def helmholtz_source(u: Separable, k: complex) -> Separable:
    """f = u_xx + u_yy + u_zz + k^2 u for a separable u (eq. (problem)).

    Each term X Y Z of u becomes four terms X''YZ, XY''Z, XYZ'', k^2 XYZ; the
    second derivatives are wrapped as factors so that further derivatives of
    f stay exact.
    """
    terms = []
    for t in u.terms:
        terms.append(Term(t.c, Shifted(t.fx, 2), t.fy, t.fz))
        terms.append(Term(t.c, t.fx, Shifted(t.fy, 2), t.fz))
        terms.append(Term(t.c, t.fx, t.fy, Shifted(t.fz, 2)))
        terms.append(Term(t.c * k * k, t.fx, t.fy, t.fz))
    return Separable(terms)


@dataclass
class Shifted(Factor):
    """The m-th derivative of another factor, as a factor of its own."""
    base: Factor
    m: int

    def d(self, x, order):
        return self.base.d(x, order + self.m)


def gaussian_sources(centres, amps, sigma: float) -> Separable:
    """Sum of isotropic Gaussians a_s exp(-|x - c_s|^2 / (2 sigma^2))."""
    terms = []
    for c, a in zip(centres, amps):
        terms.append(Term(complex(a), Gauss(c[0], sigma), Gauss(c[1], sigma), Gauss(c[2], sigma)))
    return Separable(terms)
