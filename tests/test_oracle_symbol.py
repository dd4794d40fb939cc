"""Consistency order of the interior scheme from its Fourier symbol (no GPU).

For a plane wave u = exp(i(a x + b y + c z)) the exact source is
f = (k^2 - a^2 - b^2 - c^2) u.  Inserting both into eq. (scheme) and
expanding in h must leave a residual of order h^6 (sixth-order scheme).
This pins the coefficients of (scheme), including the reading h^4/180 of
the mixed fourth-derivative term (the printed h^4/90 leaves an h^4 residual).
"""
import pytest

sp = pytest.importorskip("sympy")


def _residual(mixed_coef):
    h, a, b, c, k = sp.symbols("h a b c k", positive=True)
    # h^2 delta^2 on exp(i w x) gives -4 sin^2(w h / 2)
    sx, sy, sz = [-4 * sp.sin(w * h / 2) ** 2 for w in (a, b, c)]
    kap = k ** 2 * h ** 2
    lhs = (sx + sy + sz) / h ** 2 + (1 + kap / 30) / 6 * (sx * sy + sx * sz + sy * sz) / h ** 2 \
        + sx * sy * sz / (30 * h ** 2) + k ** 2 * (1 - kap / 12 + kap ** 2 / 360)
    xi2 = a ** 2 + b ** 2 + c ** 2
    fhat = k ** 2 - xi2
    rhs = fhat * ((1 - kap / 12 + kap ** 2 / 360) - h ** 2 / 12 * (1 - kap / 30) * xi2
                  + h ** 4 / 360 * xi2 ** 2 + mixed_coef * h ** 4 * (a**2*b**2 + a**2*c**2 + b**2*c**2))
    return sp.series(sp.expand(lhs - rhs), h, 0, 8).removeO(), h


def _lowest_order(expr, h):
    expr = sp.expand(expr)
    for p in range(0, 8):
        if sp.simplify(expr.coeff(h, p)) != 0:
            return p
    return 8


def test_interior_scheme_is_sixth_order():
    res, h = _residual(sp.Rational(1, 180))
    assert _lowest_order(res, h) >= 6


def test_printed_mixed_coefficient_would_be_fourth_order():
    res, h = _residual(sp.Rational(1, 90))
    assert _lowest_order(res, h) == 4
