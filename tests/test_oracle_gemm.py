"""Pins for the oracle's matrix products (Simple, Block, Strassen, Winograd).

What fixes the expected values here is mathematics outside the oracle:
  * integer inputs: every algorithm is exact, so the result must equal the
    integer product computed with Python integers (a wrong sign, index or
    dropped term in the Strassen / Winograd formulas, or a transposed
    operand, makes this fail);
  * the paper's benchmark matrices (Sec. 3) have a closed-form product,
    C_ij = sqrt15 n (n-1) (n + 3i - 2) / 6 (1-based i), evaluated in mpmath;
  * exact scaling by powers of two commutes with every algorithm;
  * random inputs: the row-normwise error against the exact product (itself
    pinned against Fraction in test_oracle_arith) is within the tolerance
    2^-100 l (DD) and 2^-200 l (QD).
"""
import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs

ALGS = [("simple", 0), ("block", 0), ("strassen", 1), ("strassen", 2), ("strassen", 3),
        ("winograd", 1), ("winograd", 2), ("winograd", 3)]


def rownorm_error(A, B, C, ii=None, jj=None):
    """max_i max_j |C_ij - E_ij| / max_j (|A||B|)_ij over the samples."""
    m, n = A.shape[1], B.shape[2]
    if ii is None:
        ii = np.repeat(np.arange(m), n)
        jj = np.tile(np.arange(n), m)
    err = np.abs(oracle.exact_error(A, B, C, ii, jj))
    den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)[ii]
    return float(np.max(err / den))


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (3, 5, 7), (8, 8, 8), (9, 7, 11),
                                   (16, 17, 15), (17, 16, 16), (33, 31, 30)])
def test_integer_inputs_exact_all_algorithms(P, shape):
    m, n, l = shape
    g = inputs.rng(100 + m + n + l)
    A = inputs.widen(inputs.dd_int(m, l, g), P)
    B = inputs.widen(inputs.dd_int(l, n, g), P)
    want = A[0].astype(np.int64).astype(object) @ B[0].astype(np.int64).astype(object)
    for algo, lv in ALGS:
        C = oracle.gemm(A, B, algo, lv, bs=4)
        got = sum(C[c].astype(object) for c in range(P))
        # all partial sums are integers below 2^53 * few; exact
        assert np.all(C[0].astype(object) + C[1].astype(object) == want) or \
            np.all(got == want), (algo, lv)
        assert np.all(C[0] == np.vectorize(float)(want)), (algo, lv)


def test_integer_inputs_beyond_one_double():
    """Products up to 2^80: DD must carry the low part exactly."""
    g = inputs.rng(7)
    m, n, l = 12, 10, 9
    A = inputs.dd_int(m, l, g, bound=1 << 40)
    B = inputs.dd_int(l, n, g, bound=1 << 40)
    want = A[0].astype(np.int64).astype(object) @ B[0].astype(np.int64).astype(object)
    from fractions import Fraction as F
    for algo, lv in ALGS:
        C = oracle.gemm(A, B, algo, lv, bs=4)
        for i in range(m):
            for j in range(n):
                assert F(C[0, i, j]) + F(C[1, i, j]) == want[i, j], (algo, lv, i, j)


@pytest.mark.parametrize("n", [31, 32, 33, 64])
def test_paper_matrices_closed_form(n):
    import mpmath
    A, B = inputs.paper_matrices(n)
    exact = inputs.paper_product_closed_form(n, range(n))
    for algo, lv in [("simple", 0), ("block", 0), ("strassen", 2), ("winograd", 2)]:
        C = oracle.gemm(A, B, algo, lv, bs=8)
        worst = 0
        with mpmath.workprec(300):
            for i in range(n):
                for j in (0, n // 2, n - 1):
                    got = mpmath.mpf(float(C[0, i, j])) + mpmath.mpf(float(C[1, i, j]))
                    worst = max(worst, abs(got - exact[i]) / abs(exact[i]))
        # inputs are rounded to DD (relative 2^-106 each); all terms are >= 0
        bound = (n + 4) * 2.0 ** -104 if algo in ("simple", "block") else 2.0 ** -100 * n
        assert float(worst) <= bound, (algo, float(worst) / 2.0 ** -106)


def test_power_of_two_scaling_commutes_bitwise():
    g = inputs.rng(8)
    A = inputs.dd_uniform(20, 18, g)
    B = inputs.dd_uniform(18, 22, g)
    for algo, lv in ALGS:
        C = oracle.gemm(A, B, algo, lv, bs=4)
        C2 = oracle.gemm(np.ldexp(A, 7), np.ldexp(B, -3), algo, lv, bs=4)
        assert np.array_equal(np.ldexp(C, 4), C2), algo


def test_zero_levels_is_block():
    g = inputs.rng(9)
    A = inputs.dd_uniform(13, 11, g)
    B = inputs.dd_uniform(11, 9, g)
    Cb = oracle.gemm(A, B, "block", 0, bs=4)
    for algo in ("strassen", "winograd"):
        assert np.array_equal(oracle.gemm(A, B, algo, 0, bs=4), Cb)


@pytest.mark.parametrize("shape", [(24, 24, 24), (25, 23, 27), (40, 33, 35)])
def test_dd_random_within_tolerance(shape):
    m, n, l = shape
    g = inputs.rng(10 + m)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    for algo, lv in ALGS:
        C = oracle.gemm(A, B, algo, lv, bs=8)
        e = rownorm_error(A, B, C)
        assert e <= 2.0 ** -100 * l, (algo, lv, e / 2.0 ** -106)
    # the conventional algorithms meet a much tighter, rigorous bound
    for algo in ("simple", "block"):
        assert rownorm_error(A, B, oracle.gemm(A, B, algo, 0, bs=8)) <= 4 * l * 2.0 ** -106


@pytest.mark.parametrize("shape", [(12, 12, 12), (13, 11, 15)])
def test_qd_random_within_tolerance(shape):
    m, n, l = shape
    g = inputs.rng(20 + m)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    for algo, lv in ALGS:
        C = oracle.gemm(A, B, algo, lv, bs=4)
        e = rownorm_error(A, B, C)
        assert e <= 2.0 ** -200 * l, (algo, lv)


def test_qd_of_dd_values_matches_dd_product():
    """QD inputs whose last two components are zero carry DD values; the QD
    product must agree with the DD product to DD accuracy."""
    g = inputs.rng(11)
    A = inputs.dd_uniform(10, 14, g)
    B = inputs.dd_uniform(14, 9, g)
    Cq = oracle.gemm(inputs.widen(A, 4), inputs.widen(B, 4), "winograd", 1, bs=4)
    Cd = oracle.gemm(A, B, "block", 0, bs=4)
    diff = np.abs((Cq[0] - Cd[0]) + (Cq[1] - Cd[1]) + Cq[2])
    den = np.abs(A[0]) @ np.abs(B[0])
    assert np.max(diff / den) <= 14 * 2.0 ** -104


def test_rectangular_operand_order_matters():
    """A transposed or swapped operand is caught: the product of a 3x5 by a
    5x2 integer matrix has a unique value and shape."""
    g = inputs.rng(12)
    A = inputs.dd_int(3, 5, g, bound=9)
    B = inputs.dd_int(5, 2, g, bound=9)
    C = oracle.gemm(A, B, "winograd", 2, bs=1)
    assert C.shape == (2, 3, 2)
    assert np.array_equal(C[0], A[0] @ B[0])


def test_row_scaled_inputs_keep_rownormwise_accuracy():
    """Rows of A scaled by 2^r, r in [-30, 30]: the row-normwise error of every
    algorithm stays within the tolerance (Strassen and Winograd through their
    exact equilibration), and equals the unscaled error pattern."""
    g = inputs.rng(13)
    m, n, l = 40, 36, 38
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    As, r = inputs.row_scaled(A, g)
    for algo, lv in ALGS:
        C = oracle.gemm(As, B, algo, lv, bs=8)
        e = rownorm_error(As, B, C)
        assert e <= 2.0 ** -100 * l, (algo, lv, e)
        # scaling back row i by 2^-r_i reproduces the unscaled product bitwise
        C0 = oracle.gemm(A, B, algo, lv, bs=8)
        assert np.array_equal(np.ldexp(C, -r[None, :, None]), C0), (algo, lv)
