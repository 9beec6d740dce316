"""DD Ozaki products (dd_gemm base="ozaki") at the edges of the FP64 range.

The split scales row i of A by 2^-e_i and column j of B by 2^-f_j, slices,
and scales the recombined integer sums back by 2^(e_i + f_j - 7 d).  These
cases push those exponents to their ends: all-zero rows and columns,
subnormal rows, rows and columns near 2^+-1000 (alone and against each
other), and a 2^+-100 spread of magnitudes inside one row.  Each entry must
meet the split's a-priori bound
    |C_ij - E_ij| <= l (S + 3) 2^(-7S - 2) 2^(e_i + f_j) + 2^-104 |E_ij| + 8 2^-1075
(E the exact product; the last term is the absolute resolution of a DD
number whose low part is subnormal: below 2^-968 a DD value cannot carry 106
bits, and each of the recombination's few roundings may lose half a
subnormal ulp).
"""
import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import all_entries, to_dev, to_host

pytestmark = pytest.mark.gpu

TINY = 2.0 ** -1072   # 8 times half the smallest subnormal


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def run(dd, A, B, case, **kw):
    import torch
    print(f"case ozaki range {case} A={A.shape} B={B.shape} {kw}", flush=True)
    out = dd.dd_gemm(to_dev(A), to_dev(B), base="ozaki", **kw)
    torch.cuda.synchronize()
    return to_host(out)


def scale_exp(x):
    """e with max|x| < 2^(e-1) per row of x (leading components); 1 for a
    zero row."""
    mx = np.abs(x).max(axis=1)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + 1, 1)


def check_bound(A, B, C, S=16):
    """Every entry against the a-priori bound.  The exact reference is formed
    on copies scaled by powers of two (row i of A and C by 2^s_i, column j of
    B and C by 2^t_j, bringing each row and column maximum near 1): scaling
    is exact, and the oracle's error-free products are exact only while no
    product or its error term falls below the normal range.  The bound is
    compared in the same scaled units."""
    m, n, l = A.shape[1], B.shape[2], A.shape[2]
    ii, jj = all_entries(m, n)
    ea = scale_exp(A[0])
    fb = scale_exp(B[0].T)
    s, t = 1 - ea, 1 - fb
    As = np.ldexp(A, s[None, :, None])
    Bs = np.ldexp(B, t[None, None, :])
    Cs = np.ldexp(C, (s[:, None] + t[None, :])[None])
    assert np.all(np.isfinite(C)), "non-finite output"
    err = np.abs(oracle.exact_error(As, Bs, Cs, ii, jj))
    ex = np.abs(oracle.exact_entries(As, Bs, ii, jj, kout=1)[0])
    # in scaled units 2^(e_i + f_j) becomes 4
    tiny = np.ldexp(TINY, s[ii] + t[jj])
    bound = l * (S + 3) * 2.0 ** (-7 * S) + 2.0 ** -104 * ex + tiny
    worst = float(np.max(err / bound))
    assert np.all(err <= bound), worst
    return worst


def scaled_rows(X, exps):
    """Row i of X times 2^exps[i] (exact unless it leaves the normal range)."""
    return np.ldexp(X, np.asarray(exps)[None, :, None])


@pytest.mark.parametrize("shape", [(70, 66, 75), (130, 65, 200)])
def test_zero_rows_and_columns(dd, shape):
    m, n, l = shape
    g = inputs.rng(600 + m)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    A[:, [0, 5, m - 1], :] = 0.0
    B[:, :, [1, n // 2, n - 1]] = 0.0
    # a column of B that is zero in every 32-row slab but one
    B[:, :, 9] = 0.0
    B[:, 40, 9] = [0.75, 2.0 ** -60]
    C = run(dd, A, B, "zero rows/columns")
    assert not C[:, [0, 5, m - 1], :].any()
    assert not C[:, :, [1, n // 2, n - 1]].any()
    check_bound(A, B, C)
    # with beta = 1 a zero row leaves C unchanged
    C0 = inputs.dd_uniform(m, n, g)
    import torch
    Cd = to_dev(C0)
    dd.dd_gemm(to_dev(A), to_dev(B), Cd, beta=1, base="ozaki")
    torch.cuda.synchronize()
    Ch = to_host(Cd)
    assert np.array_equal(Ch[:, [0, 5, m - 1], :], C0[:, [0, 5, m - 1], :])


def test_subnormal_rows(dd):
    m, n, l = 64, 48, 96
    g = inputs.rng(610)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    # rows 3 and 17: every entry subnormal (hi below 2^-1022, lo then zero)
    for r, e in ((3, -1040), (17, -1070)):
        A[0, r, :] = np.ldexp(A[0, r, :], e)
        A[1, r, :] = 0.0
    assert np.all(np.abs(A[0, 3]) < 2.0 ** -1022) and np.any(A[0, 17] != 0.0)
    # row 30: a few subnormal entries among normal ones
    A[0, 30, ::7] = np.ldexp(A[0, 30, ::7], -1060)
    A[1, 30, ::7] = 0.0
    C = run(dd, A, B, "subnormal rows")
    check_bound(A, B, C)
    assert np.any(C[0, 3] != 0.0)


@pytest.mark.parametrize("exp", [1000, -1000])
def test_rows_near_the_range_ends(dd, exp):
    m, n, l = 96, 70, 130
    g = inputs.rng(620)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    r = g.integers(exp - 8, exp + 1 if exp > 0 else exp + 8, m)
    A = scaled_rows(A, r)
    C = run(dd, A, B, f"rows near 2^{exp}")
    check_bound(A, B, C)


def test_rows_and_columns_at_opposite_ends(dd):
    """Rows of A near 2^1000 against columns of B near 2^-1000 (products near
    1) and rows near 2^-1000 against columns near 2^1000."""
    m, n, l = 80, 64, 100
    g = inputs.rng(630)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    ra = np.where(np.arange(m) % 2 == 0, 1000, -1000) + g.integers(-4, 5, m)
    cb = np.where(np.arange(n) % 3 == 0, -1000, 0) + g.integers(-4, 5, n)
    A = scaled_rows(A, ra)
    B = np.ldexp(B, cb[None, None, :])
    assert np.all(np.isfinite(A)) and np.all(np.isfinite(B))
    C = run(dd, A, B, "opposite ends")
    check_bound(A, B, C)


def test_wide_spread_inside_rows(dd):
    """Entries of one row spread over 2^-100 .. 2^100: the small ones fall
    below the row's slices and their contribution is within the bound."""
    m, n, l = 64, 64, 160
    g = inputs.rng(640)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    A = np.ldexp(A, g.integers(-100, 101, (m, l))[None])
    B = np.ldexp(B, g.integers(-100, 101, (l, n))[None])
    C = run(dd, A, B, "spread 2^+-100")
    check_bound(A, B, C)
    # the same matrices through the recursive form with Ozaki leaves
    import torch
    C2 = to_host(dd.dd_gemm(to_dev(A), to_dev(B), base="ozaki", algo="winograd", levels=1))
    torch.cuda.synchronize()
    ii, jj = all_entries(m, n)
    den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)
    e = np.abs(oracle.exact_error(A, B, C2, ii, jj)) / den[ii]
    assert np.max(e) <= 2.0 ** -100 * l
