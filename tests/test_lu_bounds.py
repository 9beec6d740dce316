"""Pins of the LU comparison bounds (tests/lu_bounds.py) on the CPU: two of
the oracle's own unpivoted factorizations of the paper's Sec. 4 matrix, in
different rounding orders (blocked and unblocked), meet the backward-error
bound and agree within the first-order bound; a factor entry changed in its
last bits breaks the backward-error bound.  The solve bound: the oracle's
triangular solves on given factors stay within it of the exact solution of
those factors' systems (rational arithmetic), and a solve that drops L's
low-order plane does not."""
from fractions import Fraction
import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.lu_bounds import da_bound, first_order_bound, solve_diff_bound, split, vsum

UNIT = {2: 2.0 ** -100, 4: 2.0 ** -200}


def backward_error(A, LU):
    n = A.shape[1]
    L, U = split(LU)
    ii = np.repeat(np.arange(n), n)
    jj = np.tile(np.arange(n), n)
    back = np.abs(oracle.exact_entries(L, U, ii, jj, kout=1, alpha=-1, C0=A)[0]).reshape(n, n)
    return back, da_bound(L, U, UNIT[A.shape[0]])


@pytest.mark.parametrize("P,n", [(2, 96), (4, 48)])
def test_two_oracle_factorizations_meet_the_bounds(P, n):
    A = inputs.paper_random_matrix(n, inputs.rng(0), P)
    F1, p1, i1 = oracle.getrf(A, panel=32, pivot=False, algo="block", levels=0)
    F2, p2, i2 = oracle.getrf(A, panel=1, pivot=False, algo="block", levels=0)
    assert i1 == i2 == 0
    for F in (F1, F2):
        back, bound = backward_error(A, F)
        assert np.all(back <= bound)
    L1, U1 = split(F1)
    L2, U2 = split(F2)
    tol = 2 * (first_order_bound(L1, U1, da_bound(L1, U1, UNIT[P])) +
               first_order_bound(L2, U2, da_bound(L2, U2, UNIT[P])))
    assert np.all(np.abs(vsum(F1 - F2)) <= tol)


@pytest.mark.parametrize("P", [2, 4])
def test_a_wrong_factor_entry_breaks_the_backward_bound(P):
    n = 64
    A = inputs.paper_random_matrix(n, inputs.rng(1), P)
    F, _, _ = oracle.getrf(A, panel=16, pivot=False, algo="block", levels=0)
    for (i, j) in ((40, 7), (7, 40)):          # a multiplier, then an entry of U
        G = F.copy()
        G[P - 1, i, j] = G[P - 1, i, j] + np.ldexp(abs(G[0, i, j]), -70 if P == 2 else -160)
        back, bound = backward_error(A, G)
        assert np.any(back > bound), (i, j)


def exact_lu_solve(LU, ipiv, b):
    """x with L U x = P b exactly (rationals): the interchanges replayed on b,
    then forward and back substitution."""
    P, n = LU.shape[0], LU.shape[1]
    F = [[sum(Fraction(float(LU[c, i, j])) for c in range(P)) for j in range(n)] for i in range(n)]
    y = [sum(Fraction(float(b[c, i, 0])) for c in range(P)) for i in range(n)]
    for k in range(n):
        p = int(ipiv[k])
        y[k], y[p] = y[p], y[k]
    for i in range(n):
        y[i] -= sum(F[i][j] * y[j] for j in range(i))
    x = [Fraction(0)] * n
    for i in reversed(range(n)):
        x[i] = (y[i] - sum(F[i][j] * x[j] for j in range(i + 1, n))) / F[i][i]
    return x


@pytest.mark.parametrize("P,u", [(2, 2.0 ** -104), (4, 2.0 ** -208)])
def test_solve_bound_holds_for_the_oracle_solve_and_fails_without_a_plane(P, u):
    n = 16
    g = inputs.rng(5)
    A = inputs.paper_random_matrix(n, g, P)
    LU, ipiv, _ = oracle.getrf(A, panel=4, pivot=True, algo="block", levels=0)
    b = np.zeros((P, n, 1))
    b[0, :, 0] = g.uniform(-1, 1, n)
    x = exact_lu_solve(LU, ipiv, b)
    xg = oracle.getrs(LU, ipiv, b)
    bound = solve_diff_bound(LU, xg, u)[:, 0]
    err = np.array([float(sum(Fraction(float(xg[c, i, 0])) for c in range(P)) - x[i])
                    for i in range(n)])
    assert np.all(np.abs(err) <= bound / 2)      # one solve: half of the two-solve bound
    assert np.any(bound > 0)
    # the same solve with the low-order planes of L's multipliers dropped
    bad = LU.copy()
    low = np.tril(np.ones((n, n), dtype=bool), -1)
    bad[1:, low] = 0.0
    xb = oracle.getrs(bad, ipiv, b)
    diff = np.abs(vsum(xb - xg))[:, 0]
    assert np.any(diff > solve_diff_bound(LU, xg, u)[:, 0])


def block_inverse_solve(T, b, lower, block):
    """X := T^-1 b by blocks in FP64: each diagonal block's inverse formed by
    substitution on the unit vectors, applied to the block's residual."""
    from scipy.linalg import solve_triangular
    n = T.shape[0]
    x = b.astype(np.float64).copy()
    starts = list(range(0, n, block))
    for i0 in (starts if lower else starts[::-1]):
        i1 = min(n, i0 + block)
        r = x[i0:i1] - (T[i0:i1, :i0] @ x[:i0] if lower else T[i0:i1, i1:] @ x[i1:])
        Z = solve_triangular(T[i0:i1, i0:i1], np.eye(i1 - i0), lower=lower, unit_diagonal=lower)
        x[i0:i1] = Z @ r
    return x


def test_block_inverse_solve_bound():
    """The block term: a block-inverse solve in FP64 (u = 2^-53) stays within
    the block solve's half of the bound of the exact rational solution of the
    same factors; a block solve that ignores the multipliers inside its
    diagonal blocks breaks it."""
    n, block = 24, 8
    g = inputs.rng(7)
    A = inputs.paper_random_matrix(n, g, 2)
    F, ipiv, _ = oracle.getrf(A, panel=4, pivot=True, algo="block", levels=0)
    LU = F[:1].copy()                        # FP64 factors: the leading plane
    b = np.zeros((1, n, 1))
    b[0, :, 0] = g.uniform(-1, 1, n)
    x = np.array([float(v) for v in exact_lu_solve(LU, ipiv, b)])
    L, U = split(LU)
    pb = b[0, :, 0].copy()
    for k in range(n):
        p = int(ipiv[k])
        pb[k], pb[p] = pb[p], pb[k]
    u = 2.0 ** -53
    xb = block_inverse_solve(U[0], block_inverse_solve(L[0], pb, True, block), False, block)
    full = solve_diff_bound(LU, x[None, :, None], u, block=block)[:, 0]
    sub = solve_diff_bound(LU, x[None, :, None], u)[:, 0] / 2   # the substitution half
    assert np.all(np.abs(xb - x) <= full - sub)
    # a wrong block solve: the multipliers inside the diagonal blocks dropped
    Lw = L[0].copy()
    for i0 in range(0, n, block):
        Lw[i0:i0 + block, i0:i0 + block] = np.eye(block)
    xw = block_inverse_solve(U[0], block_inverse_solve(Lw, pb, True, block), False, block)
    assert np.any(np.abs(xw - x) > full)
