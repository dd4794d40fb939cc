"""GPU right-hand-side assembly for separable sources and nonhomogeneous
Dirichlet data (include/helmholtz6.h: helmholtz6_rhs_separable,
helmholtz6_rhs_dirichlet_z), compared element by element with the oracle's
F, then used to run the paper's 3D experiments with F built on the device:
Table 3 and Table 5 (errors and counts at h = 1/64 .. 1/256) and the
h = 1/512 rows of Tables 6 and 8 (1.3e8 unknowns; the oracle cannot build F
there), and the psi rows of Tables 4, 6 and 8 (eq. (PSI)).

The factor samples handed to the device are evaluations of the manufactured
solutions (problem inputs); the source terms, face terms and plane coupling
are computed by the kernels.  FP64 throughout: the same terms summed in a
different order, so the F comparison allows 1e-12 relative to max |F|."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from manufactured import (cuda_values, face_tables, factor_tables, mixed_pattern_u, neumann_data_y_u,
                          neumann_data_z_u, neumann_y_factor, normal_derivative, source, table3_u, table5_u,
                          sommerfeld_z_factor)
from oracle.functions import Cos, Poly, Separable, Sin, Term

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.fixture(scope="module")
def h6():
    from paper_1212_1397_amd import helmholtz6
    return helmholtz6


def table8_u(k):
    return Separable([Term(1.0, Poly((0, 0, 0, 1, -3, 3, -1)), Poly((0, 1, -1)) * Cos(k * math.pi),
                           sommerfeld_z_factor(k))])


def neumann_box_u(k):
    """Neumann x and y pairs, Neumann at z = 0 and data at z = 1: exercises the
    mirror rule of the Dirichlet plane term and every Neumann face term."""
    return Separable([Term(0.7 - 0.2j, neumann_y_factor(), Cos(2 * math.pi), Cos(k * math.pi) + Poly((0, 0, 1))),
                      Term(0.3, Cos(math.pi), neumann_y_factor(), Cos(k * math.pi))])


def gpu_rhs(h6, plan, prob, u, k, top_data):
    f = source(u, k)
    coef, tx, ty, tz = factor_tables(f, prob.points())
    F = plan.rhs_separable(coef, tx, ty, tz)
    if top_data:
        x, y, _ = prob.points()
        g = cuda_values(u, (x, y, np.array([prob.length(2)])))[0].contiguous()
        plan.rhs_dirichlet_z(1, g, F)
    return F


CASES = [
    ("DDDDDD", (14, 11, 9), 20.0, table3_u, False),
    ("DDDDND", (10, 12, 13), 20.0, table5_u, True),
    ("DDNNSS", (9, 10, 12), 12.0 + 0.4j, mixed_pattern_u, False),
    ("DDDDSS", (12, 9, 10), 7.0 - 0.3j, table8_u, False),
    ("NNNNND", (9, 11, 8), 6.0, neumann_box_u, True),
]


@pytest.mark.parametrize("bc,n,k,ufun,top", CASES)
def test_separable_rhs_matches_oracle(h6, bc, n, k, ufun, top):
    h = 1.0 / (max(n) + 1)
    prob = oracle.Problem(n, h, complex(k), tuple(bc))
    u = ufun(k)
    ref = oracle.rhs(prob, source(u, k), dirichlet_z=(None, u) if top else (None, None))
    plan = h6.Plan(n, h, k, bc)
    F = gpu_rhs(h6, plan, prob, u, k, top).cpu().numpy()
    err = np.abs(F - ref).max() / np.abs(ref).max()
    print(f"{bc} n = {n}: max |F_gpu - F_oracle| / max |F| = {err:.2e}", flush=True)
    assert err < 1e-12


def test_rhs_zero_terms_and_scaling(h6):
    """nterms = 0 gives F = 0; F is linear in the term coefficients."""
    prob = oracle.Problem((8, 9, 10), 1 / 11, 5.0 + 0j, tuple("DDNNSS"))
    plan = h6.Plan(prob.n, prob.h, prob.k, "DDNNSS")
    F0 = plan.rhs_separable([], *[np.zeros((0, 5, d)) for d in plan.dims])
    assert torch.count_nonzero(F0) == 0
    coef, tx, ty, tz = factor_tables(source(mixed_pattern_u(5.0), 5.0), prob.points())
    F1 = plan.rhs_separable(coef, tx, ty, tz)
    F2 = plan.rhs_separable(2.5j * coef, tx, ty, tz)
    assert float(torch.linalg.norm(F2 - 2.5j * F1) / torch.linalg.norm(F1)) < 1e-14


def run_table(h6, ufun, bc, H, top, k=20.0):
    prob = oracle.Problem.cube(H - 1, k, bc)
    u = ufun(k)
    plan = h6.Plan(prob.n, prob.h, k, bc)
    F = gpu_rhs(h6, plan, prob, u, k, top)
    ex = cuda_values(u, prob.points())
    U, info = plan.solve(F, method="gmres", restart=30, tol=1e-10, maxit=300)
    Us, infs = plan.solve(F, method="sks", tol=1e-10, maxit=300)
    e6 = float((U - ex).abs().max())
    e6s = float((Us - ex).abs().max())
    plan.close()
    return e6, e6s, info["iters"], infs["iters"]


@pytest.mark.parametrize("i", [0, 1, 2])
def test_table3_on_device(h6, i):
    t = GOLD["table3"]
    H = t["h"][i]
    e6, e6s, ng, ns = run_table(h6, table3_u, "DDDDDD", H, False)
    print(f"Table 3, h = 1/{H}: err GMRES {e6:.3e}, SKS {e6s:.3e} (printed {t['err6'][i]:.3e}); "
          f"GMRES {ng} ({t['gmres'][i]}), SKS {ns} ({t['sks'][i]})", flush=True)
    assert abs(e6 - t["err6"][i]) <= 0.015 * t["err6"][i]
    assert abs(e6s - t["err6"][i]) <= 0.015 * t["err6"][i]
    assert ns == t["sks"][i] and abs(ng - t["gmres"][i]) <= 2


@pytest.mark.parametrize("i", [0, 1, 2])
def test_table5_on_device(h6, i):
    t = GOLD["table5"]
    H = t["h"][i]
    e6, e6s, ng, ns = run_table(h6, table5_u, "DDDDND", H, True)
    print(f"Table 5, h = 1/{H}: err GMRES {e6:.3e}, SKS {e6s:.3e} (printed {t['err6'][i]:.3e}); "
          f"GMRES {ng} ({t['gmres'][i]}), SKS {ns} ({t['sks'][i]})", flush=True)
    assert abs(e6 - t["err6"][i]) <= 0.015 * t["err6"][i]
    assert abs(e6s - t["err6"][i]) <= 0.015 * t["err6"][i]
    assert ns == t["sks"][i] and abs(ng - t["gmres"][i]) <= 2


def counts_512(h6, ufun, bc, k, top):
    prob = oracle.Problem.cube(511, k, bc)
    u = ufun(k)
    plan = h6.Plan(prob.n, prob.h, k, bc)
    F = gpu_rhs(h6, plan, prob, u, k, top)
    out = {}
    for m in ("gmres", "sks"):
        kw = dict(tol=1e-10, maxit=100)
        if m == "gmres":
            kw["restart"] = 10
        _, info = plan.solve(F, method=m, **kw)
        out[m] = info
    plan.close()
    del F
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("ki", [0, 1, 2, 3, 4])
def test_table6_h512(h6, ki):
    """Table 6, h = 1/512 (511 x 511 x 512 unknowns): SKS counts exact.  GMRES
    is reported only: the printed counts come from left-preconditioned GMRES
    stopped on the preconditioned residual, ours from right preconditioning
    stopped on the true residual."""
    t = GOLD["table6"]
    k = float(t["k"][ki])
    g, s = t["rows"]["512"][ki]
    c = counts_512(h6, table5_u, "DDDDND", k, True)
    print(f"Table 6, h = 1/512, k = {k}: GMRES {c['gmres']['iters']} ({g}), "
          f"SKS {c['sks']['iters']} {c['sks']['status']} ({s})", flush=True)
    assert c["gmres"]["status"] == "ok"
    assert c["sks"]["status"] == "ok" and c["sks"]["iters"] == s


@pytest.mark.parametrize("ki", [0, 1, 2, 3, 4, 5])
def test_table8_h512(h6, ki):
    """Table 8, h = 1/512: the consistent Sommerfeld test function replaces the
    printed one, so SKS counts are compared within 2; GMRES reported."""
    t = GOLD["table8"]
    kk = t["k"][ki]
    k = complex(kk[0], kk[1]) if isinstance(kk, list) else complex(kk)
    g, s = t["rows"]["512"][ki]
    c = counts_512(h6, table8_u, "DDDDSS", k, False)
    print(f"Table 8, h = 1/512, k = {k}: GMRES {c['gmres']['iters']} ({g}), "
          f"SKS {c['sks']['iters']} {c['sks']['status']} ({s})", flush=True)
    assert c["gmres"]["status"] == "ok"
    assert c["sks"]["status"] == "ok" and abs(c["sks"]["iters"] - s) <= 2


def sks_residuals(h6, ufun, bc, H, k, top):
    """(||r_0||, ||r_1||, ||r_2||) / ||F|| of Algorithm 1: r_0 = F, then the
    residuals of the first two iterations of the loop (the solver's history
    holds the relative residuals after each iteration)."""
    prob = oracle.Problem.cube(H - 1, k, bc)
    plan = h6.Plan(prob.n, prob.h, k, bc)
    F = gpu_rhs(h6, plan, prob, ufun(k), k, top)
    _, info = plan.solve(F, method="sks", tol=0.0, maxit=2)
    plan.close()
    return (1.0, info["history"][0], info["history"][1])


PSI_TABLES = {"table4": (table3_u, "DDDDDD", False), "table6": (table5_u, "DDDDND", True),
              "table8": (table8_u, "DDDDSS", False)}


@pytest.mark.parametrize("table", ["table4", "table6", "table8"])
def test_psi_rows(h6, table):
    """eq. (PSI) with gamma = 2 from the first two SKS iterations on h = 1/256
    and h = 1/128, the grids the paper uses for every psi row.  Table 4
    (Dirichlet) is held to its printed row within 0.2.  The Dirichlet-Neumann
    and Dirichlet-Sommerfeld rows (Tables 6, 8) are not reproduced, under
    this reading (||r_2|| / ||r_1||) or with ||r_1|| / ||r_0||, so they are
    reported; what is checked there is the paper's conclusion from them,
    psi > 0 (convergence improves as h decreases)."""
    ufun, bc, top = PSI_TABLES[table]
    t = GOLD[table]
    got = []
    for kk in t["k"]:
        k = complex(kk[0], kk[1]) if isinstance(kk, list) else complex(kk)
        fine = sks_residuals(h6, ufun, bc, 256, k, top)
        coarse = sks_residuals(h6, ufun, bc, 128, k, top)
        got.append(h6.psi_order(fine[1], fine[2], coarse[1], coarse[2], 2.0))
    print(f"{table} psi: " + ", ".join(f"{g:.2f} ({p})" for g, p in zip(got, t["psi"])), flush=True)
    for g, p in zip(got, t["psi"]):
        assert g > 0
        if table == "table4":
            assert abs(g - p) < 0.2


def neumann_data_x_u():
    return Separable([Term(0.8 + 0.3j, Sin(math.pi / 2), Sin(math.pi), Sin(2 * math.pi)),
                      Term(0.4, Cos(math.pi) * Poly((0.5, 1.0)), Sin(2 * math.pi), Sin(math.pi))])


NEUMANN_CASES = [
    ("DDDDND", (10, 12, 13), 7.0, neumann_data_z_u, (4,)),
    ("DDNNDD", (9, 11, 10), 5.0 + 0.2j, neumann_data_y_u, (2, 3)),
    ("NNDDSS", (12, 9, 10), 6.0 + 0.1j, neumann_data_x_u, (0, 1)),
]


def gpu_rhs_with_neumann(plan, prob, u, k, faces):
    coef, tx, ty, tz = factor_tables(source(u, k), prob.points())
    F = plan.rhs_separable(coef, tx, ty, tz)
    for face in faces:
        ax, side = divmod(face, 2)
        g = normal_derivative(u, ax)
        c, t1, t2 = face_tables(g, prob.points(), ax, 0.0 if side == 0 else prob.length(ax))
        plan.rhs_neumann(face, c, t1, t2, F)
    return F


@pytest.mark.parametrize("bc,n,k,ufun,faces", NEUMANN_CASES)
def test_neumann_data_rhs_matches_oracle(h6, bc, n, k, ufun, faces):
    """Nonzero Neumann data (eq. (3DN)) on z, y and x faces: device F equals the oracle's."""
    h = 1.0 / (max(n) + 1)
    prob = oracle.Problem(n, h, complex(k), tuple(bc))
    u = ufun()
    ref = oracle.rhs(prob, source(u, k), neumann={f: normal_derivative(u, f // 2) for f in faces})
    plan = h6.Plan(n, h, k, bc)
    F = gpu_rhs_with_neumann(plan, prob, u, k, faces).cpu().numpy()
    err = np.abs(F - ref).max() / np.abs(ref).max()
    print(f"{bc} faces {faces}: max |F_gpu - F_oracle| / max |F| = {err:.2e}", flush=True)
    assert err < 1e-12
    with pytest.raises(h6.H6Error):
        plan.rhs_neumann(5 if bc[5] != "N" else 4 if bc[4] != "N" else 0, *face_tables(
            normal_derivative(u, 2), prob.points(), 2, 0.0), torch.zeros_like(torch.from_numpy(ref)).cuda())


def test_neumann_data_solution_is_sixth_order(h6):
    """With nonzero u_z on the Neumann face, GPU solutions on F built on the
    device converge at sixth order (error ratio about 64 per halving of h)."""
    k = 10.0
    u = neumann_data_z_u()
    errs = []
    for n in (15, 31, 63):
        prob = oracle.Problem.cube(n, k, "DDDDND")
        plan = h6.Plan(prob.n, prob.h, k, "DDDDND")
        F = gpu_rhs_with_neumann(plan, prob, u, k, (4,))
        U, info = plan.solve(F, method="gmres", restart=30, tol=1e-12, maxit=300)
        assert info["status"] == "ok"
        errs.append(float((U - cuda_values(u, prob.points())).abs().max()))
        plan.close()
    r = [errs[i] / errs[i + 1] for i in range(2)]
    print(f"errors {errs}, ratios {r}", flush=True)
    assert all(56 <= x <= 72 for x in r), r
