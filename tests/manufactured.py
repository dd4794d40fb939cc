"""Manufactured solutions used by the oracle tests (exact u, f = lap u + k^2 u)."""
import math

from oracle.functions import Cos, Exp, Poly, Separable, Shifted, Sin, Term, helmholtz_source


def table3_u(k):
    """Section 4.2.1: u = x^3(1-x)^3 * y(1-y)cos(k pi y) * sin(k pi z)."""
    return Separable([Term(1.0, Poly((0, 0, 0, 1, -3, 3, -1)),
                           Poly((0, 1, -1)) * Cos(k * math.pi), Sin(k * math.pi))])


def table5_u(k):
    """Section 4.2.2: as Table 3 with cos(k pi z) (u_z = 0 at z = 0, u = u_b at z = 1)."""
    return Separable([Term(1.0, Poly((0, 0, 0, 1, -3, 3, -1)),
                           Poly((0, 1, -1)) * Cos(k * math.pi), Cos(k * math.pi))])


def neumann_z_u():
    """u_z(0) = 0, u(1) = 0 and u_zzz(0) != 0, so the Neumann source terms are active."""
    return Separable([Term(1.0, Sin(math.pi), Sin(2 * math.pi), Cos(math.pi / 2) * Poly((1, 0, 0, 1)))])


def neumann_y_factor():
    """Y'(0) = Y'(1) = 0 and Y'''(0) = -12: an active Neumann pair on y."""
    return Cos(math.pi) + Poly((0, 0, 1, -2, 1))


def sommerfeld_z_factor(k):
    """psi(z) = e^{-ikz}(1 + c z^2), c = ik/(1 - ik): u_z + iku = 0 at z = 0 and
    u_z - iku = 0 at z = 1 (the printed test function of Table 7 satisfies only
    the second condition, so it is not used)."""
    c = 1j * k / (1 - 1j * k)
    return Exp(-1j * k) * Poly((1, 0, c))


def mixed_pattern_u(k):
    """x Dirichlet, y Neumann, z Sommerfeld: the face pattern of the benchmark grids."""
    return Separable([Term(1.0, Sin(math.pi), neumann_y_factor(), sommerfeld_z_factor(k))])


def source(u, k):
    return helmholtz_source(u, k)


def factor_tables(f, pts):
    """Inputs of helmholtz6_rhs_separable for a separable f: the term
    coefficients and, per axis, the derivatives of orders 0..4 of each
    factor at the unknown nodes pts = (x, y, z)."""
    import numpy as np
    coef = np.array([t.c for t in f.terms], dtype=np.complex128)
    tabs = [np.stack([np.stack([getattr(t, fa).d(p, o) for o in range(5)]) for t in f.terms])
            for fa, p in zip(("fx", "fy", "fz"), pts)]
    return (coef, *tabs)


def cuda_values(u, pts, device="cuda"):
    """u at the tensor grid pts as a complex128 CUDA tensor of shape
    (len(z), len(y), len(x)), built term by term on the device."""
    import numpy as np
    import torch
    x, y, z = pts
    out = torch.zeros((len(z), len(y), len(x)), dtype=torch.complex128, device=device)
    for t in u.terms:
        X = torch.from_numpy(np.asarray(t.fx.d(x, 0), dtype=np.complex128)).to(device)
        Y = torch.from_numpy(np.asarray(t.fy.d(y, 0), dtype=np.complex128)).to(device)
        Z = torch.from_numpy(np.asarray(t.fz.d(z, 0), dtype=np.complex128)).to(device)
        out += t.c * Z[:, None, None] * Y[None, :, None] * X[None, None, :]
    return out


def normal_derivative(u, ax):
    """du/d(axis ax) as a separable function: Neumann data of u on that axis' faces."""
    out = []
    for t in u.terms:
        fs = [t.fx, t.fy, t.fz]
        fs[ax] = Shifted(fs[ax], 1)
        out.append(Term(t.c, *fs))
    return Separable(out)


def neumann_data_z_u():
    """u_z(x, y, 0) = pi sin(pi x) sin(2 pi y) != 0, u = 0 on the other faces."""
    return Separable([Term(1.0, Sin(math.pi), Sin(2 * math.pi), Sin(math.pi))])


def neumann_data_y_u():
    """u_y(x, 0, z) = (pi/2) sin(pi x) sin(2 pi z) != 0, u_y(x, 1, z) = 0."""
    return Separable([Term(1.0, Sin(math.pi), Sin(math.pi / 2), Sin(2 * math.pi))])


def face_tables(g, pts, ax, coord):
    """Inputs of helmholtz6_rhs_neumann for data g (separable) on the face
    axis ax = coord: per term the coefficient times the normal factor's value
    on the face, and derivative tables (orders 0..4) along the two tangential
    axes (increasing order) at the unknown nodes pts."""
    import numpy as np
    ta, tb = [a for a in range(3) if a != ax]
    coef, t1, t2 = [], [], []
    for t in g.terms:
        fs = [t.fx, t.fy, t.fz]
        coef.append(t.c * complex(np.asarray(fs[ax].d(np.array([coord]), 0))[0]))
        t1.append(np.stack([fs[ta].d(pts[ta], o) for o in range(5)]))
        t2.append(np.stack([fs[tb].d(pts[tb], o) for o in range(5)]))
    return np.array(coef, dtype=np.complex128), np.stack(t1), np.stack(t2)
