"""The one-dimensional model problem of Section 2 (Dirichlet, unit interval).

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle; it exists to
reproduce Table 2 and the closed-form eigenvalues of Theorem 3.

Scheme (Section 2, derived from (T1D) and (T2D)), h = 1/(N+1):
  d1 U_{i-1} + d2 U_i + d1 U_{i+1} = F_i,
  d1 = 1 - k^4 h^4 / 360,   d2 = -2 + k^2 h^2 - 7 k^4 h^4 / 90,
  F_i = h^2 (1 - 7 k^2 h^2 / 90) f_i - (k^2 h^4 / 360)(f_{i-1} + f_{i+1})
        + (7 h^4 / 90) f''_i + (h^4 / 360)(f''_{i-1} + f''_{i+1}).
The printed F_i carries k^4 h^4 where the derivation from (T2D) gives
k^2 h^2 (first term) and k^2 h^4 (second term); the derived form is used.
Preconditioner (1DAP): A_p = Lambda - (2 - k^2 h^2) I.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


class OneD:
    def __init__(self, N: int, k: complex):
        self.N, self.k = N, complex(k)
        self.h = 1.0 / (N + 1)
        self.kap = (self.k * self.h) ** 2
        self.d1 = 1.0 - self.kap ** 2 / 360.0
        self.d2 = -2.0 + self.kap - 7.0 * self.kap ** 2 / 90.0
        self.x = np.arange(1, N + 1) * self.h

    def apply_A(self, U):
        out = self.d2 * U
        out[1:] += self.d1 * U[:-1]
        out[:-1] += self.d1 * U[1:]
        return out

    def apply_Ap(self, U):
        out = -(2.0 - self.kap) * U
        out[1:] += U[:-1]
        out[:-1] += U[1:]
        return out

    def apply_Pinv(self, R):
        """A_p^{-1} by the sine transform: eigenvalues -4 sin^2(j pi h/2) + k^2 h^2."""
        M = self.N + 1
        lam = -4.0 * np.sin(np.arange(1, self.N + 1) * np.pi / (2 * M)) ** 2 + self.kap
        c = sfft.dst(np.asarray(R, dtype=np.complex128), type=1) / M
        return 0.5 * sfft.dst(c / lam, type=1)

    def rhs(self, f, f2):
        """F from callables f and f'' (values on the closed grid x_0..x_{N+1})."""
        h, kap = self.h, self.kap
        xx = np.arange(0, self.N + 2) * h
        fv, f2v = f(xx), f2(xx)
        return (h * h * (1.0 - 7.0 * kap / 90.0) * fv[1:-1]
                - (kap * h * h / 360.0) * (fv[:-2] + fv[2:])
                + (7.0 * h ** 4 / 90.0) * f2v[1:-1]
                + (h ** 4 / 360.0) * (f2v[:-2] + f2v[2:]))

    def eigenvalues(self):
        """Theorem 3: lambda_j = -4 sin^2(j pi h/2) + h^2k^2 - h^4k^4 (14 + cos(j pi h))/180."""
        j = np.arange(1, self.N + 1)
        return (-4.0 * np.sin(j * np.pi * self.h / 2.0) ** 2 + self.kap
                - self.kap ** 2 * (14.0 + np.cos(j * np.pi * self.h)) / 180.0)
