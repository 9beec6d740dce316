"""GPU parity of the CRT INT8-MFMA base (dd_gemm base="crt").

The base rounds row i of A (scaled by 2^-e_i, max|a_ik| < 2^(e_i - 1)) and
column j of B (2^-f_j) to integers of P1 = 107 bits, multiplies their
residues modulo N pairwise coprime moduli exactly on INT8 matrix cores and
rebuilds the integer product by the Chinese remainder theorem in 160-bit
fixed point.  Bars, per entry against the exact product E (oracle):
    |C_ij - E_ij| <= (l (2^P1 + 1) + N 128 M 2^-160) 2^(e_i + f_j - 2 P1)
                     + 2^-103 |E_ij|
(the first term: each operand moved by at most one unit of its integer; the
second: the rebuild's fixed-point truncation; the last: the DD rounding of
the result), and the row-normwise tolerance 2^-100 l of the other bases.
Integer inputs need no rounding: the leading component of every entry is
then the exact integer.  The edge cases of the FP64 range are those of the
Ozaki split's tests, against this bound.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import (all_entries, rownorm_den, rownorm_error, sample_entries, to_dev,
                           to_host, value_diff)

pytestmark = pytest.mark.gpu

P1 = 107
TINY = 2.0 ** -1072   # 8 times half the smallest subnormal (see the Ozaki range tests)


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def run(dd, A, B, C0=None, case="", **kw):
    import torch
    print(f"case crt {case} A={A.shape} B={B.shape} {kw}", flush=True)
    out = dd.dd_gemm(to_dev(A), to_dev(B), to_dev(C0) if C0 is not None else None, base="crt",
                     **kw)
    torch.cuda.synchronize()
    return to_host(out)


def scale_exp(x):
    """e with max|x| < 2^(e-1) per row of x (leading components); 1 for a
    zero row."""
    mx = np.abs(x).max(axis=1)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + 1, 1)


def unit_terms(dd, l):
    """l (2^P1 + 1) + N 128 M 2^-160, in units of 2^(e_i + f_j - 2 P1)."""
    ms = dd.crt_moduli(l)
    M = math.prod(ms)
    return l * (2.0 ** P1 + 1) + len(ms) * 128 * (M / 2.0 ** 160)


def check_bound(dd, A, B, C, alpha=1, C0=None):
    """Every entry against the a-priori bound.  The exact reference is formed
    on copies scaled by powers of two (row i of A and C by 2^s_i, column j of
    B and C by 2^t_j, bringing each row and column maximum near 1), where the
    oracle's error-free products stay in the normal range; the bound is
    compared in the same scaled units (2^(e_i + f_j) becomes 4)."""
    m, n, l = A.shape[1], B.shape[2], A.shape[2]
    ii, jj = all_entries(m, n)
    ea = scale_exp(A[0])
    fb = scale_exp(B[0].T)
    s, t = 1 - ea, 1 - fb
    As = np.ldexp(A, s[None, :, None])
    Bs = np.ldexp(B, t[None, None, :])
    Cs = np.ldexp(C, (s[:, None] + t[None, :])[None])
    C0s = None if C0 is None else np.ldexp(C0, (s[:, None] + t[None, :])[None])
    assert np.all(np.isfinite(C)), "non-finite output"
    err = np.abs(oracle.exact_error(As, Bs, Cs, ii, jj, alpha=alpha, C0=C0s))
    ex = np.abs(oracle.exact_entries(As, Bs, ii, jj, kout=1, alpha=alpha, C0=C0s)[0])
    tiny = np.ldexp(TINY, s[ii] + t[jj])
    bound = unit_terms(dd, l) * 4.0 * 2.0 ** (-2 * P1) + 2.0 ** -103 * ex + tiny
    if C0 is not None:  # the DD addition of C0
        bound = bound + 2.0 ** -104 * (ex + np.abs(C0s[0][ii, jj]))
    worst = float(np.max(err / bound))
    assert np.all(err <= bound), worst
    return worst


@pytest.mark.parametrize("shape", [(1, 1, 1), (32, 32, 32), (63, 65, 67), (128, 128, 128),
                                   (129, 130, 131), (200, 1, 77), (3, 300, 500),
                                   (257, 140, 96)])
def test_random_dd_vs_oracle_and_bound(dd, shape):
    m, n, l = shape
    g = inputs.rng(880 + m + n)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, case="random")
    ii, jj = all_entries(m, n)
    den = rownorm_den(A, B)
    e = rownorm_error(A, B, C, ii, jj, den=den)
    assert e <= 2.0 ** -100 * l, e
    check_bound(dd, A, B, C)
    Co = oracle.gemm(A, B, "block")
    d = float(np.max(value_diff(C, Co) / den[:, None]))
    assert d <= 2 * 2.0 ** -100 * l, d


@pytest.mark.parametrize("shape", [(9, 7, 11), (64, 64, 64), (130, 100, 257)])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1), ("strassen", 2)])
def test_integer_inputs(dd, shape, algo, lv):
    """Integers need no rounding; what remains is the rebuild's and the
    result's DD rounding (relative to a leaf's result, which the recursive
    forms' additions may cancel): the leading components are the exact
    product (an integer below 2^53, the error far below 1/2) and the
    trailing ones within the row-normwise tolerance."""
    m, n, l = shape
    g = inputs.rng(870 + m)
    A = inputs.dd_int(m, l, g)
    B = inputs.dd_int(l, n, g)
    C = run(dd, A, B, case="integers", algo=algo, levels=lv)
    E = A[0] @ B[0]
    assert np.array_equal(C[0], E)
    den = rownorm_den(A, B)
    assert np.all(np.abs(C[1]) <= 2.0 ** -100 * l * den[:, None])


@pytest.mark.parametrize("alpha,beta", [(1, 1), (-1, 1), (-1, 0)])
def test_alpha_beta(dd, alpha, beta):
    g = inputs.rng(890)
    m, n, l = 70, 45, 53
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C0 = inputs.dd_uniform(m, n, g)
    C = run(dd, A, B, C0=C0, case="alpha/beta", alpha=alpha, beta=beta)
    ii, jj = all_entries(m, n)
    e = rownorm_error(A, B, C, ii, jj, alpha=alpha, C0=C0 if beta else None)
    assert e <= 2.0 ** -100 * l, e
    check_bound(dd, A, B, C, alpha=alpha, C0=C0 if beta else None)


@pytest.mark.parametrize("algo,lv", [("winograd", 1), ("strassen", 2), ("winograd", 3)])
def test_recursive_forms_on_crt_leaves(dd, algo, lv):
    g = inputs.rng(895 + lv)
    m, n, l = 300, 260, 280
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, case="recursive", algo=algo, levels=lv)
    ii, jj = all_entries(m, n)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -100 * l


def test_long_k_uses_several_exact_chunks(dd):
    """l > 65536 K values per exact INT32 product: two chunks, the second
    added to C in DD."""
    g = inputs.rng(893)
    m, n, l = 40, 36, 66000
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, case="long K")
    ii, jj = sample_entries(m, n, 40)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -100 * l


def test_equal_accuracy_with_fma(dd):
    n = 1024
    g = inputs.rng(1)
    A = inputs.dd_uniform(n, n, g)
    B = inputs.dd_uniform(n, n, g)
    As, _ = inputs.row_scaled(A, g)
    ii, jj = sample_entries(n, n, 300)
    for X in (A, As):
        Cc = run(dd, X, B, case="n=1024")
        Cf = to_host(dd.dd_gemm(to_dev(X), to_dev(B), base="fma"))
        ec = rownorm_error(X, B, Cc, ii, jj)
        ef = rownorm_error(X, B, Cf, ii, jj)
        assert ec <= 2.0 ** -100 * n and ef <= 2.0 ** -100 * n
        assert ec <= 16 * ef + 2.0 ** -104, (ec, ef)


@pytest.mark.parametrize("n", [1024, 2048])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1)])
def test_full_size_sampled(dd, n, algo, lv):
    g = inputs.rng(0)
    A = inputs.dd_uniform(n, n, g)
    B = inputs.dd_uniform(n, n, g)
    C = run(dd, A, B, case="full size", algo=algo, levels=lv)
    ii, jj = sample_entries(n, n, 200)
    e = rownorm_error(A, B, C, ii, jj)
    assert e <= 2.0 ** -100 * n, e


def test_deterministic(dd):
    """A Winograd level's 7 leaves run as one batched CRT product; the same
    level computed again gives the same bits."""
    g = inputs.rng(896)
    A = inputs.dd_uniform(256, 192, g)
    B = inputs.dd_uniform(192, 224, g)
    C1 = run(dd, A, B, case="deterministic", algo="winograd", levels=1)
    C2 = run(dd, A, B, case="deterministic", algo="winograd", levels=1)
    assert np.array_equal(C1, C2)


# ---- the ends of the FP64 range ------------------------------------------------

def test_zero_rows_and_columns(dd):
    m, n, l = 130, 65, 200
    g = inputs.rng(900)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    A[:, [0, 5, m - 1], :] = 0.0
    B[:, :, [1, n // 2, n - 1]] = 0.0
    B[:, :, 9] = 0.0
    B[:, 40, 9] = [0.75, 2.0 ** -60]
    C = run(dd, A, B, case="zero rows/columns")
    assert not C[:, [0, 5, m - 1], :].any()
    assert not C[:, :, [1, n // 2, n - 1]].any()
    check_bound(dd, A, B, C)


def test_subnormal_rows(dd):
    m, n, l = 64, 48, 96
    g = inputs.rng(910)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    for r, e in ((3, -1040), (17, -1070)):
        A[0, r, :] = np.ldexp(A[0, r, :], e)
        A[1, r, :] = 0.0
    A[0, 30, ::7] = np.ldexp(A[0, 30, ::7], -1060)
    A[1, 30, ::7] = 0.0
    C = run(dd, A, B, case="subnormal rows")
    check_bound(dd, A, B, C)
    assert np.any(C[0, 3] != 0.0)


@pytest.mark.parametrize("exp", [1000, -1000])
def test_rows_near_the_range_ends(dd, exp):
    m, n, l = 96, 70, 130
    g = inputs.rng(920)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    r = g.integers(exp - 8, exp + 1 if exp > 0 else exp + 8, m)
    A = np.ldexp(A, r[None, :, None])
    C = run(dd, A, B, case=f"rows near 2^{exp}")
    check_bound(dd, A, B, C)


def test_rows_and_columns_at_opposite_ends(dd):
    m, n, l = 80, 64, 100
    g = inputs.rng(930)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    ra = np.where(np.arange(m) % 2 == 0, 1000, -1000) + g.integers(-4, 5, m)
    cb = np.where(np.arange(n) % 3 == 0, -1000, 0) + g.integers(-4, 5, n)
    A = np.ldexp(A, ra[None, :, None])
    B = np.ldexp(B, cb[None, None, :])
    C = run(dd, A, B, case="opposite ends")
    check_bound(dd, A, B, C)


def test_wide_spread_inside_rows(dd):
    m, n, l = 64, 64, 160
    g = inputs.rng(940)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    A = np.ldexp(A, g.integers(-100, 101, (m, l))[None])
    B = np.ldexp(B, g.integers(-100, 101, (l, n))[None])
    C = run(dd, A, B, case="spread 2^+-100")
    check_bound(dd, A, B, C)


# ---- LU with CRT trailing updates -----------------------------------------------

@pytest.mark.parametrize("n,panel", [(300, 64), (1024, 128)])
def test_lu_with_crt_updates(dd, n, panel):
    """The factorization's trailing updates on the CRT base (partial
    pivoting on a matrix without a boosted diagonal): the solve's residual,
    formed exactly by the oracle, within n 2^-100."""
    import torch
    print(f"case crt lu n={n} panel={panel}", flush=True)
    g = inputs.rng(950 + n)
    A = inputs.dd_lu_matrix(n, g, boost=False)
    LU = to_dev(A)
    ipiv, perm, info = dd.dd_getrf(LU, panel=panel, algo="winograd", levels=1, base="crt")
    B = inputs.dd_uniform(n, 2, g)
    X = to_dev(B)
    dd.dd_getrs(LU, ipiv, X, perm=perm)
    torch.cuda.synchronize()
    assert int(to_host(info)[0]) == 0
    assert oracle.lu_residual(A, to_host(X), B) <= n * 2.0 ** -100
