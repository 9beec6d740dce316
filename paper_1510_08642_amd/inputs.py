"""Seeded synthetic inputs for DD/QD matrix products and DD LU.

This module only draws numbers: it holds none of the DD/QD arithmetic of the
method.  Every generator returns float64 arrays in *plane layout*
(``(P, rows, cols)``: P = 2 for DD, 4 for QD, component 0 the largest), and
every multi-component number it returns is already non-overlapping, built by
exponent manipulation alone (``frexp`` / ``ldexp``), so neither side has to
renormalise it.

Recipes (numpy ``default_rng(seed)``, PCG64):
  * DD uniform: hi ~ U[-1, 1), lo = ulp(hi)/2 * U(-1, 1) (|lo| < ulp(hi)/2).
  * QD uniform: c0 ~ U[-1, 1); c_k = ulp(c_{k-1})/2 * (+-U[1/2, 1)), random
    signs, so the trailing terms sit about 2^-54, 2^-108, 2^-162 below c0.
  * DD LU matrix: hi ~ N(0, 1) plus n on the diagonal, lo as above.
  * Integer matrices: integer hi, zero lo (products and sums stay exact).
  * The paper's benchmark matrices (Sec. 3): A = [sqrt5 (i + j - 1)],
    B = [sqrt3 (n - i)], each entry the DD nearest to the real value,
    computed with mpmath at 300 bits.
  * Row scaling by powers of two (exact).
"""
from __future__ import annotations

import numpy as np


def _half_ulp_scaled(x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """u * ulp(x)/2 with |u| < 1, for float64 x (0 where x == 0)."""
    _, e = np.frexp(x)                  # x = f * 2^e, f in [1/2, 1)
    out = np.ldexp(u, e - 54)           # ulp(x) = 2^(e-53)
    return np.where(x == 0.0, 0.0, out)


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def dd_from_hi(hi: np.ndarray, g: np.random.Generator) -> np.ndarray:
    """Attaches a random low part below half an ulp to each hi."""
    hi = np.asarray(hi, dtype=np.float64)
    lo = _half_ulp_scaled(hi, g.uniform(-1.0, 1.0, hi.shape))
    return np.stack([hi, lo])


def dd_uniform(rows: int, cols: int, g: np.random.Generator) -> np.ndarray:
    return dd_from_hi(g.uniform(-1.0, 1.0, (rows, cols)), g)


def qd_uniform(rows: int, cols: int, g: np.random.Generator) -> np.ndarray:
    c = [g.uniform(-1.0, 1.0, (rows, cols))]
    for _ in range(3):
        mag = g.uniform(0.5, 1.0, (rows, cols))
        sgn = np.where(g.random((rows, cols)) < 0.5, -1.0, 1.0)
        c.append(_half_ulp_scaled(c[-1], sgn * mag))
    return np.stack(c)


def qd_lu_matrix(n: int, g: np.random.Generator, boost: bool = True) -> np.ndarray:
    """QD version of dd_lu_matrix: leading term N(0, 1) (+ n on the diagonal),
    trailing terms as in qd_uniform."""
    c = [g.standard_normal((n, n))]
    if boost:
        c[0][np.arange(n), np.arange(n)] += float(n)
    for _ in range(3):
        mag = g.uniform(0.5, 1.0, (n, n))
        sgn = np.where(g.random((n, n)) < 0.5, -1.0, 1.0)
        c.append(_half_ulp_scaled(c[-1], sgn * mag))
    return np.stack(c)


def dd_lu_matrix(n: int, g: np.random.Generator, boost: bool = True) -> np.ndarray:
    hi = g.standard_normal((n, n))
    if boost:
        hi[np.arange(n), np.arange(n)] += float(n)
    return dd_from_hi(hi, g)


def dd_int(rows: int, cols: int, g: np.random.Generator, bound: int = 1 << 20) -> np.ndarray:
    hi = g.integers(-bound, bound + 1, (rows, cols)).astype(np.float64)
    return np.stack([hi, np.zeros_like(hi)])


def widen(X: np.ndarray, P: int) -> np.ndarray:
    """Pads a plane-layout matrix with zero planes up to P components."""
    if X.shape[0] >= P:
        return X[:P].copy()
    return np.concatenate([X, np.zeros((P - X.shape[0],) + X.shape[1:])])


def row_scaled(X: np.ndarray, g: np.random.Generator, lo: int = -30, hi: int = 30):
    """Multiplies row i by 2^r_i, r_i uniform integers in [lo, hi] (exact)."""
    r = g.integers(lo, hi + 1, X.shape[1])
    return np.ldexp(X, r[None, :, None]), r


def _mp_terms(v, P: int) -> tuple:
    """The first P terms of v, each the double nearest the remaining value."""
    import mpmath
    out = []
    for _ in range(P):
        h = float(v)
        out.append(h)
        v = v - mpmath.mpf(h)
    return tuple(out)


def _mp_dd(v) -> tuple[float, float]:
    return _mp_terms(v, 2)


def paper_matrices(n: int, P: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """A = [sqrt5 (i+j-1)], B = [sqrt3 (n-i)], 1-based, as DD (P = 2) or QD
    (P = 4) numbers nearest the real values (Sec. 3)."""
    import mpmath
    with mpmath.workprec(400):
        s5, s3 = mpmath.sqrt(5), mpmath.sqrt(3)
        a_vals = np.array([_mp_terms(s5 * t, P) for t in range(1, 2 * n)])        # i+j-1
        b_vals = np.array([_mp_terms(s3 * (n - i), P) for i in range(1, n + 1)])  # n-i
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    A = np.stack([a_vals[i + j, c] for c in range(P)])
    B = np.stack([np.broadcast_to(b_vals[:, c][:, None], (n, n)) for c in range(P)]).copy()
    return A, B


def paper_product_closed_form(n: int, rows) -> list:
    """mpmath values of C_ij = sqrt15 n (n-1) (n + 3i - 2) / 6 (1-based i),
    the exact product of the paper's matrices; independent of j."""
    import mpmath
    with mpmath.workprec(400):
        s15 = mpmath.sqrt(15)
        return [s15 * n * (n - 1) * (n + 3 * (int(r) + 1) - 2) / 6 for r in rows]


def paper_random_matrix(n: int, g: np.random.Generator, P: int = 2) -> np.ndarray:
    """The Sec. 4 random matrix: entries uniform in [-1, 1] as DD (P = 2) or QD
    (P = 4) numbers (lower parts below half an ulp of the part above)."""
    return dd_uniform(n, n, g) if P == 2 else qd_uniform(n, n, g)


def serving_trace(nreq: int, rate: float, seed: int = 0, gemm_frac: float = 0.6,
                  gemm_n=(64, 1024), lu_n=(128, 2048), nrhs=(1, 16)):
    """Poisson arrivals mixing DD GEMM and DD LU-solve requests.

    Sizes are log-uniform in the given ranges.  Returns a list of dicts with
    keys kind ('gemm' | 'lu'), n, nrhs, t_arrive (seconds), seed."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, nreq))
    out = []
    for k in range(nreq):
        if g.random() < gemm_frac:
            n = int(round(np.exp(g.uniform(np.log(gemm_n[0]), np.log(gemm_n[1])))))
            out.append(dict(kind="gemm", n=n, nrhs=0, t_arrive=float(t[k]), seed=int(k)))
        else:
            n = int(round(np.exp(g.uniform(np.log(lu_n[0]), np.log(lu_n[1])))))
            r = int(g.integers(nrhs[0], nrhs[1] + 1))
            out.append(dict(kind="lu", n=n, nrhs=r, t_arrive=float(t[k]), seed=int(k)))
    return out
