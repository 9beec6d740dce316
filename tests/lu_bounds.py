"""Bounds for comparing two LU factorizations computed in different rounding
orders (used by the LU parity tests): the backward error elimination
guarantees, and the first-order perturbation bound of the factors."""
import numpy as np


def split(LU):
    """Unit lower L and upper U of a plane-layout factorization."""
    P, n = LU.shape[0], LU.shape[1]
    low = np.tril(np.ones((n, n), dtype=bool), -1)
    L = np.where(low[None], LU, 0.0)
    L[0][np.arange(n), np.arange(n)] = 1.0
    U = np.where(~low[None], LU, 0.0)
    return L, U


def da_bound(L, U, u):
    """Entrywise bound on the backward error of factors L, U (leading parts)."""
    n = L.shape[1]
    aL, aU = np.abs(L[0]), np.abs(U[0])
    comp = aL @ aU
    rowcol = aL.max(axis=1)[:, None] * aU.max(axis=0)[None, :]
    return n * u * np.maximum(comp, rowcol)


def first_order_bound(L, U, dA):
    from scipy.linalg import solve_triangular
    n = L.shape[1]
    Li = np.abs(solve_triangular(L[0], np.eye(n), lower=True, unit_diagonal=True))
    Ui = np.abs(solve_triangular(U[0], np.eye(n), lower=False))
    X = Li @ dA @ Ui
    upper = np.triu(np.ones((n, n), dtype=bool))
    return np.where(upper, np.triu(X) @ np.abs(U[0]), np.abs(L[0]) @ np.tril(X, -1))


def samples(n, count, seed):
    g = np.random.default_rng(seed)
    ii = np.concatenate([np.arange(n), [0, n - 1], g.integers(0, n, count)])
    jj = np.concatenate([np.arange(n), [n - 1, 0], g.integers(0, n, count)])
    return ii, jj


def vsum(X):
    return sum(X[c] for c in range(X.shape[0]))


def _block_term(T, block):
    """|D| |D^-1| |D| |D^-1| |D| + |D| |D^-1| |D| for the block diagonal D of T
    (blocks of `block` rows): the backward error a block solve adds when it
    applies a computed inverse of its diagonal block."""
    from scipy.linalg import block_diag
    n = T.shape[0]
    Ds, Di = [], []
    for i0 in range(0, n, block):
        D = T[i0:i0 + block, i0:i0 + block]
        Ds.append(np.abs(D))
        Di.append(np.abs(np.linalg.inv(D)))
    aD, aDi = block_diag(*Ds), block_diag(*Di)
    return aD @ aDi @ aD @ aDi @ aD + aD @ aDi @ aD


def solve_diff_bound(LU, x, u, block=None):
    """Componentwise bound on the difference of two solutions of L U x = P b
    by triangular solves on the same factors, each backward stable with
    |dL| <= n u |L|, |dU| <= n u |U| (any summation order): to first order
    |x_hat - x| <= n u (|U^-1| |U| |x| + |U^-1| |L^-1| |L| |U x|) for each, so
    twice that for two (FP64 inverses; a further factor 2 covers their
    relative error).  With `block`, one of the two solves applies computed
    inverses Z = D^-1 + E of the diagonal blocks (|E| <= n u |D^-1||D||D^-1|,
    the columns of Z found by substitution) to the block residuals r = D x:
    that adds D (E r + e) to the backward error of each block, bounded by
    n u (|D||D^-1||D||D^-1| + |D||D^-1|) |D| |x|, i.e. the term
    _block_term(T) |x| beside |T| |x| for each triangle T."""
    from scipy.linalg import solve_triangular
    L, U = split(LU)
    n = L.shape[1]
    x0 = vsum(x) if x.ndim == 3 else x
    Li = np.abs(solve_triangular(L[0], np.eye(n), lower=True, unit_diagonal=True))
    Ui = np.abs(solve_triangular(U[0], np.eye(n), lower=False))
    aL, aU = np.abs(L[0]), np.abs(U[0])
    y = np.abs(U[0] @ x0)
    one = Ui @ (aU @ np.abs(x0)) + Ui @ (Li @ (aL @ y))
    if block is None:
        return 4 * n * u * one
    extra = Ui @ (_block_term(U[0], block) @ np.abs(x0)) + Ui @ (Li @ (_block_term(L[0], block) @ y))
    return 2 * n * u * one + 2 * n * u * (one + extra)
