"""Pins of the oracle's operators against closed forms and an independent
row-by-row assembly (no GPU)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle.precond import forward_transform, inverse_transform, mode_eigenvalues
from dense_assembly import dense_A, dense_Ap

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))

BC_CASES = ["DDDDDD", "DDNNSS", "NNNNNN", "NNDDSN", "DDDDND", "DDDDSD", "NNNNSS", "DDNNDN"]


def _sine_mode(prob, i, j, l):
    x, y, z = prob.points()
    return (np.sin(l * np.pi * z)[:, None, None] * np.sin(j * np.pi * y)[None, :, None]
            * np.sin(i * np.pi * x)[None, None, :]) + 0j


@pytest.mark.parametrize("k", [3.0, 7.5 + 0.4j, 19.0])
def test_dirichlet_eigenmodes_of_A_and_Ap(k):
    """Section 3.4 (3DEGV): sine modes are eigenvectors with closed-form eigenvalues."""
    prob = oracle.Problem.cube(9, k)
    for (i, j, l) in [(1, 1, 1), (1, 2, 3), (9, 4, 2), (5, 9, 9), (7, 1, 6)]:
        v = _sine_mode(prob, i, j, l)
        lam = oracle.dirichlet_eigenvalue(prob, i, j, l)
        lamp = oracle.dirichlet_eigenvalue_p(prob, i, j, l)
        Av = oracle.apply_A(prob, v)
        assert np.abs(Av - lam * v).max() <= 1e-13 * np.abs(v).max() * max(1.0, abs(lam))
        Apv = oracle.apply_Ap(prob, v)
        assert np.abs(Apv - lamp * v).max() <= 1e-13 * np.abs(v).max() * max(1.0, abs(lamp))


def test_table1_eigenvalue_bounds():
    """Table 1: bounds of 1 - lambda/lambda^p over all Dirichlet modes, h = 1/(N+1)."""
    t1 = GOLD["table1"]
    for H, row in t1["rows"].items():
        H = int(H)
        r = np.arange(1, H)
        for k, (m_pr, M_pr) in zip(t1["k"], row):
            p = oracle.Problem.cube(H - 1, float(k))
            I, J, L = np.meshgrid(r, r, r, indexing="ij", sparse=True)
            q = (1.0 - oracle.dirichlet_eigenvalue(p, I, J, L) / oracle.dirichlet_eigenvalue_p(p, I, J, L)).real
            m, M = float(q.min()), float(q.max())
            assert abs(m - m_pr) <= 0.02 * abs(m_pr), (H, k, m, m_pr)
            assert abs(M - M_pr) <= 0.02 * abs(M_pr), (H, k, M, M_pr)


@pytest.mark.parametrize("bc", BC_CASES)
def test_matrix_free_equals_row_assembly(bc):
    """The composition form equals the 27-point row-by-row assembly with explicit closures."""
    prob = oracle.Problem((4, 3, 5), 1.0 / 6.5, 7.0 + 0.6j, tuple(bc))
    A = dense_A(prob)
    Ap = dense_Ap(prob)
    N = A.shape[0]
    cols = np.eye(N, dtype=np.complex128)
    Am = np.stack([oracle.apply_A(prob, cols[j].reshape(prob.shape)).ravel() for j in range(N)], 1)
    Apm = np.stack([oracle.apply_Ap(prob, cols[j].reshape(prob.shape)).ravel() for j in range(N)], 1)
    assert np.abs(A - Am).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(Ap - Apm).max() <= 1e-14 * np.abs(Ap).max()


def test_dirichlet_operator_is_complex_symmetric():
    prob = oracle.Problem.cube(4, 6.0 + 1.0j)
    A = dense_A(prob)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()


@pytest.mark.parametrize("code,L", [("D", 7), ("N", 9), ("D", 1), ("N", 3)])
def test_transform_pair_matches_explicit_eigenbasis(code, L):
    """W^{-1} and W of Section 3.3 against explicitly built sine/cosine matrices."""
    if code == "D":
        M = L + 1
        q = np.arange(1, L + 1)
        W = np.sin(np.pi * np.outer(q, q) / M)
    else:
        M = L - 1
        q = np.arange(0, L)
        W = np.cos(np.pi * np.outer(q, q) / M)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    c = forward_transform(r, 0, code)
    assert np.allclose(W @ c, r, atol=1e-14, rtol=0)
    assert np.allclose(inverse_transform(c, 0, code), r, atol=1e-14, rtol=0)
    # columns of W are eigenvectors of the 1D block with eigenvalue -4 sin^2(pi m / 2M)
    T = -2.0 * np.eye(L) + np.eye(L, k=1) + np.eye(L, k=-1)
    if code == "N":
        T[0, 1] = T[-1, -2] = 2.0
    m = q
    lam = -4.0 * np.sin(np.pi * m / (2 * M)) ** 2
    assert np.allclose(T @ W, W * lam[None, :], atol=1e-13)


@pytest.mark.parametrize("bc", BC_CASES)
def test_Pinv_inverts_Ap(bc):
    prob = oracle.Problem((5, 4, 6), 1.0 / 7.0, 8.0 + 0.3j, tuple(bc))
    rng = np.random.default_rng(1)
    r = rng.standard_normal(prob.shape) + 1j * rng.standard_normal(prob.shape)
    z = oracle.apply_Pinv(prob, r)
    assert np.abs(oracle.apply_Ap(prob, z) - r).max() <= 1e-13 * np.abs(r).max()
    Ap = dense_Ap(prob)
    z2 = np.linalg.solve(Ap, r.ravel())
    assert np.abs(z.ravel() - z2).max() <= 1e-12 * np.abs(z2).max()


def test_singular_preconditioner_detected():
    """k^2 h^2 on the 7-point spectrum: the (1,1,1) mode of A_p vanishes."""
    n = 8
    h = 1.0 / (n + 1)
    kap = 12.0 * np.sin(np.pi * h / 2) ** 2
    prob = oracle.Problem.cube(n, np.sqrt(kap) / h)
    with pytest.raises(oracle.SingularPreconditioner):
        oracle.apply_Pinv(prob, np.ones(prob.shape, dtype=np.complex128))


def test_unsupported_faces_rejected():
    with pytest.raises(oracle.UnsupportedBC):
        oracle.Problem.cube(4, 1.0, "SSDDDD")
    with pytest.raises(oracle.UnsupportedBC):
        oracle.Problem.cube(4, 1.0, "DDDNDD")
