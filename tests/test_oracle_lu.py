"""Pins for the oracle's blocked DD LU (Sec. 4) and solve (Eq. 2).

Expected values come from structure, not from the oracle: diagonal and
triangular matrices have known exact factors; a permutation matrix has known
pivots; an integer A = L U with unit-lower L and power-of-two pivots is
recovered exactly; a small random case is compared with LU in exact rational
arithmetic; and the paper's test solution x = [0, 1, ..., n-1] (Sec. 4) gives a
forward error that must sit near DD precision for a well-conditioned A.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs


def dd(hi):
    hi = np.asarray(hi, dtype=np.float64)
    return np.stack([hi, np.zeros_like(hi)])


@pytest.mark.parametrize("pivot", [False, True])
def test_diagonal_and_upper_triangular_exact(pivot):
    g = inputs.rng(30)
    n = 19
    D = np.diag(g.uniform(1, 2, n))
    LU, ipiv, info = oracle.getrf(dd(D), panel=4, pivot=pivot, algo="winograd", levels=1)
    assert info == 0 and np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(LU[0], D) and not LU[1].any()
    Up = np.triu(g.uniform(-1, 1, (n, n))) + np.diag(np.full(n, 4.0))
    LU, ipiv, info = oracle.getrf(dd(Up), panel=5, pivot=pivot, algo="strassen", levels=1)
    # below-diagonal zeros divide to zero, updates subtract exact zeros
    assert np.array_equal(LU[0], Up) and not LU[1].any()


def test_permutation_matrix_pivots():
    n = 11
    perm = np.array([3, 0, 7, 1, 10, 2, 5, 9, 4, 6, 8])
    Pm = np.zeros((n, n))
    Pm[np.arange(n), perm] = 1.0
    LU, ipiv, info = oracle.getrf(dd(Pm), panel=3, pivot=True, algo="block")
    assert info == 0
    # replay the interchanges on the identity's row order: must give Pm's rows
    rows = list(range(n))
    for i, p in enumerate(ipiv):
        rows[i], rows[p] = rows[p], rows[i]
    assert np.array_equal(Pm[rows], np.eye(n))
    assert np.array_equal(LU[0], np.eye(n))


@pytest.mark.parametrize("algo,levels", [("block", 0), ("strassen", 2), ("winograd", 2)])
def test_integer_factors_recovered_exactly(algo, levels):
    g = inputs.rng(31)
    n = 24
    L = np.tril(g.integers(-3, 4, (n, n)), -1) + np.eye(n, dtype=np.int64)
    d = 2.0 ** g.integers(-2, 3, n)
    U = np.triu(g.integers(-3, 4, (n, n)), 1).astype(np.float64) + np.diag(d)
    A = L.astype(np.float64) @ U
    LU, ipiv, info = oracle.getrf(dd(A), panel=8, pivot=False, algo=algo, levels=levels)
    assert info == 0
    assert np.array_equal(np.tril(LU[0], -1), np.tril(L, -1).astype(np.float64))
    assert np.array_equal(np.triu(LU[0]), U)
    assert not LU[1].any()


def test_singular_info():
    A = np.ones((6, 6))
    A[0, 0] = 2.0
    LU, ipiv, info = oracle.getrf(dd(A), panel=2, pivot=True, algo="block")
    # column 0 pivots on 2, column 1 on 1/2, then column 2 (1-based 3) is all zero
    assert info == 3


def test_random_small_against_rational_lu():
    g = inputs.rng(32)
    n = 12
    A = inputs.dd_lu_matrix(n, g, boost=False)
    LU, ipiv, info = oracle.getrf(A, panel=4, pivot=True, algo="winograd", levels=1)
    Af = [[F(A[0, i, j]) + F(A[1, i, j]) for j in range(n)] for i in range(n)]
    # the exact partial-pivoting choice must agree with the oracle's
    M = [row[:] for row in Af]
    for c in range(n):
        p = max(range(c, n), key=lambda r: (abs(M[r][c]), -r))
        assert p == ipiv[c]
        M[c], M[p] = M[p], M[c]
        for r in range(c + 1, n):
            M[r][c] = M[r][c] / M[c][c]
            for cc in range(c + 1, n):
                M[r][cc] -= M[r][c] * M[c][cc]
    scale = max(abs(x) for row in M for x in row)
    for i in range(n):
        for j in range(n):
            got = F(LU[0, i, j]) + F(LU[1, i, j])
            assert abs(got - M[i][j]) <= scale * F(2) ** -96


@pytest.mark.parametrize("algo,levels,panel", [("block", 0, 16), ("winograd", 1, 16),
                                                ("winograd", 2, 32), ("strassen", 1, 24)])
def test_paper_solution_forward_error_and_residual(algo, levels, panel):
    g = inputs.rng(33)
    n = 96
    A = inputs.dd_lu_matrix(n, g)
    x = dd(np.arange(n, dtype=np.float64)[:, None])
    b = oracle.exact_entries(A, x, np.arange(n), np.zeros(n, dtype=np.int64), kout=2)
    b = b.reshape(2, n, 1)
    LU, ipiv, info = oracle.getrf(A, panel=panel, pivot=True, algo=algo, levels=levels)
    X = oracle.getrs(LU, ipiv, b)
    rel = [abs((F(X[0, i, 0]) + F(X[1, i, 0]) - i) / i) for i in range(1, n)]
    assert float(max(rel)) <= n * 2.0 ** -100
    assert oracle.lu_residual(A, X, b) <= n * 2.0 ** -100


def test_winograd_update_error_close_to_block():
    """The paper finds no visible error increase from the Winograd update on
    a random matrix (Sec. 4); here: within a factor of 16 of Block's."""
    g = inputs.rng(34)
    n = 80
    A = inputs.dd_lu_matrix(n, g, boost=False)
    x = dd(np.arange(n, dtype=np.float64)[:, None])
    b = oracle.exact_entries(A, x, np.arange(n), np.zeros(n, dtype=np.int64), kout=2).reshape(2, n, 1)
    errs = {}
    for algo, lv in [("block", 0), ("winograd", 2)]:
        LU, ipiv, _ = oracle.getrf(A, panel=16, pivot=True, algo=algo, levels=lv)
        X = oracle.getrs(LU, ipiv, b)
        errs[algo] = oracle.lu_residual(A, X, b)
    assert errs["winograd"] <= 16 * errs["block"] + n * 2.0 ** -106


# ---- QD (the paper's second LU workload, Sec. 4 with QD arithmetic) --------

def qd(hi):
    hi = np.asarray(hi, dtype=np.float64)
    return np.stack([hi] + [np.zeros_like(hi)] * 3)


def fq(x):
    return sum(F(float(c)) for c in x)


@pytest.mark.parametrize("algo,levels", [("block", 0), ("winograd", 2)])
def test_qd_integer_factors_recovered_exactly(algo, levels):
    g = inputs.rng(35)
    n = 20
    L = np.tril(g.integers(-3, 4, (n, n)), -1) + np.eye(n, dtype=np.int64)
    d = 2.0 ** g.integers(-2, 3, n)
    U = np.triu(g.integers(-3, 4, (n, n)), 1).astype(np.float64) + np.diag(d)
    A = L.astype(np.float64) @ U
    LU, ipiv, info = oracle.getrf(qd(A), panel=8, pivot=False, algo=algo, levels=levels)
    assert info == 0
    assert np.array_equal(np.tril(LU[0], -1), np.tril(L, -1).astype(np.float64))
    assert np.array_equal(np.triu(LU[0]), U)
    assert not LU[1:].any()


def test_qd_random_small_against_rational_lu():
    g = inputs.rng(36)
    n = 10
    A = inputs.qd_lu_matrix(n, g, boost=False)
    LU, ipiv, info = oracle.getrf(A, panel=4, pivot=True, algo="winograd", levels=1)
    M = [[fq(A[:, i, j]) for j in range(n)] for i in range(n)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: (abs(M[r][c]), -r))
        assert p == ipiv[c]
        M[c], M[p] = M[p], M[c]
        for r in range(c + 1, n):
            M[r][c] = M[r][c] / M[c][c]
            for cc in range(c + 1, n):
                M[r][cc] -= M[r][c] * M[c][cc]
    scale = max(abs(x) for row in M for x in row)
    for i in range(n):
        for j in range(n):
            assert abs(fq(LU[:, i, j]) - M[i][j]) <= scale * F(2) ** -196


def test_qd_pivot_decided_below_the_leading_term():
    """Candidates whose leading terms are equal: the second and third terms
    decide, as the exact comparison does."""
    n = 8
    A = qd(np.eye(n) * 0.25)
    A[:, :, 0] = 0.0
    A[0, [2, 5, 6], 0] = [1.0, 1.0, -1.0]
    A[1, [2, 5, 6], 0] = [2.0 ** -60, 2.0 ** -60, -(2.0 ** -60)]
    A[2, [2, 5, 6], 0] = [2.0 ** -120, 2.0 ** -118, -(2.0 ** -119)]
    LU, ipiv, info = oracle.getrf(A, panel=4, pivot=True, algo="block")
    assert ipiv[0] == 5


@pytest.mark.parametrize("algo,levels,panel", [("block", 0, 16), ("winograd", 1, 16)])
def test_qd_paper_solution_forward_error_and_residual(algo, levels, panel):
    g = inputs.rng(37)
    n = 48
    A = inputs.qd_lu_matrix(n, g)
    x = qd(np.arange(n, dtype=np.float64)[:, None])
    b = oracle.exact_entries(A, x, np.arange(n), np.zeros(n, dtype=np.int64), kout=4)
    b = b.reshape(4, n, 1)
    LU, ipiv, info = oracle.getrf(A, panel=panel, pivot=True, algo=algo, levels=levels)
    X = oracle.getrs(LU, ipiv, b)
    rel = [abs((fq(X[:, i, 0]) - i) / i) for i in range(1, n)]
    assert float(max(rel)) <= n * 2.0 ** -196
    assert oracle.lu_residual(A, X, b) <= n * 2.0 ** -200
