"""GPU parity of the QD Ozaki INT8-MFMA base (qd_gemm base="ozaki").

Bars: integer inputs exact (small integers bit-exact, integers beyond one
double exact as values); random QD within the QD row-normwise tolerance
2^-200 l at the default S = 31 and, per entry, within the method's a-priori
bound
    |C_ij - E_ij| <= l (S + 3) 2^(-7S - 2) 2^(e_i + f_j) + 2^-208 |E_ij|
for every supported S (e_i, f_j the scaling exponents: max|a_ik| < 2^(e_i-1));
agreement with the oracle's QD Block product and with the FMA base.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import (all_entries, rownorm_den, rownorm_error, sample_entries, to_dev,
                           to_host, value_diff)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def run(dd, A, B, C0=None, **kw):
    import torch
    print(f"case qd ozaki A={A.shape} B={B.shape} {kw}", flush=True)
    out = dd.qd_gemm(to_dev(A), to_dev(B), to_dev(C0) if C0 is not None else None,
                     base="ozaki", **kw)
    torch.cuda.synchronize()
    return to_host(out)


def scale_exp(x):
    mx = np.abs(x).max(axis=1)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + 1, 1)


def apriori_ok(A, B, C, ii, jj, S, alpha=1, C0=None):
    l = A.shape[2]
    err = np.abs(oracle.exact_error(A, B, C, ii, jj, alpha=alpha, C0=C0))
    ea = scale_exp(A[0])
    fb = scale_exp(B[0].T)
    ex = np.abs(oracle.exact_entries(A, B, ii, jj, kout=1, alpha=alpha, C0=C0)[0])
    bound = l * (S + 3) * np.ldexp(1.0, -7 * S - 2 + ea[ii] + fb[jj]) + 2.0 ** -208 * ex
    return bool(np.all(err <= bound)), float(np.max(err / bound))


def qd_from_ints(V):
    """Integers below 2^100 as exact two-term values in QD planes."""
    hi = np.array([[float(v) for v in row] for row in V])
    lo = np.array([[float(v - int(h)) for v, h in zip(row, hrow)] for row, hrow in zip(V, hi)])
    z = np.zeros_like(hi)
    return np.stack([hi, lo, z, z])


@pytest.mark.parametrize("shape", [(9, 7, 11), (64, 64, 64), (65, 66, 67), (130, 100, 257)])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1), ("strassen", 2)])
def test_integer_inputs_bit_exact(dd, shape, algo, lv):
    m, n, l = shape
    g = inputs.rng(170 + m)
    A = inputs.widen(inputs.dd_int(m, l, g), 4)
    B = inputs.widen(inputs.dd_int(l, n, g), 4)
    C = run(dd, A, B, algo=algo, levels=lv)
    assert np.array_equal(C[0], A[0] @ B[0])
    assert not C[1:].any()


def test_integer_inputs_beyond_two_doubles(dd):
    """70-bit integers: products of 140 bits, sums needing three doubles; every
    digit and every diagonal is kept, so the value is exact."""
    g = np.random.default_rng(171)
    m, n, l = 33, 40, 45
    Ai = [[int(g.integers(-(1 << 62), 1 << 62)) * 256 + int(g.integers(0, 256))
           for _ in range(l)] for _ in range(m)]
    Bi = [[int(g.integers(-(1 << 62), 1 << 62)) * 256 + int(g.integers(0, 256))
           for _ in range(n)] for _ in range(l)]
    A, B = qd_from_ints(Ai), qd_from_ints(Bi)
    C = run(dd, A, B)
    for i in range(0, m, 4):
        for j in range(0, n, 3):
            want = sum(Ai[i][k] * Bi[k][j] for k in range(l))
            assert sum(F(C[c, i, j]) for c in range(4)) == want, (i, j)


@pytest.mark.parametrize("shape", [(1, 1, 1), (32, 32, 32), (31, 33, 65), (70, 66, 75),
                                   (129, 97, 130), (3, 200, 97), (200, 1, 40)])
def test_random_qd_vs_oracle_and_bound(dd, shape):
    m, n, l = shape
    g = inputs.rng(180 + m + n)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B)
    ii, jj = all_entries(m, n)
    den = rownorm_den(A, B)
    e = rownorm_error(A, B, C, ii, jj, den=den)
    assert e <= 2.0 ** -200 * l, e
    ok, worst = apriori_ok(A, B, C, ii, jj, 31)
    assert ok, worst
    Co = oracle.gemm(A, B, "block")
    d = float(np.max(value_diff(C, Co) / den[:, None]))
    assert d <= 2 * 2.0 ** -200 * l, d


@pytest.mark.parametrize("alpha,beta", [(1, 1), (-1, 1), (-1, 0)])
def test_alpha_beta(dd, alpha, beta):
    g = inputs.rng(190)
    m, n, l = 70, 45, 53
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C0 = inputs.qd_uniform(m, n, g)
    C = run(dd, A, B, C0=C0, alpha=alpha, beta=beta)
    ii, jj = all_entries(m, n)
    e = rownorm_error(A, B, C, ii, jj, alpha=alpha, C0=C0 if beta else None)
    assert e <= 2.0 ** -200 * l, e


@pytest.mark.parametrize("S", [28, 29, 30, 31])
def test_slice_count_meets_apriori_bound(dd, S):
    g = inputs.rng(191)
    m, n, l = 96, 80, 150
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B, slices=S)
    ii, jj = all_entries(m, n)
    ok, worst = apriori_ok(A, B, C, ii, jj, S)
    assert ok, (S, worst)


def test_more_slices_is_more_accurate(dd):
    g = inputs.rng(192)
    m, n, l = 64, 64, 256
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    ii, jj = all_entries(m, n)
    errs = [rownorm_error(A, B, run(dd, A, B, slices=S), ii, jj) for S in (28, 29, 30)]
    assert all(errs[i + 1] < errs[i] / 16 for i in range(len(errs) - 1)), errs


def test_unsupported_slice_count_is_an_error(dd):
    import torch
    g = inputs.rng(193)
    A = to_dev(inputs.qd_uniform(8, 8, g))
    with pytest.raises(RuntimeError):
        dd.qd_gemm(A, A, base="ozaki", slices=20)
    torch.cuda.synchronize()


def test_long_k_uses_several_exact_chunks(dd):
    """l > 16384 K values per exact INT32 accumulation: two chunks."""
    g = inputs.rng(194)
    m, n, l = 40, 36, 17000
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B)
    ii, jj = sample_entries(m, n, 40)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -200 * l
    g2 = inputs.rng(195)
    Ai = inputs.widen(inputs.dd_int(m, l, g2, bound=1 << 10), 4)
    Bi = inputs.widen(inputs.dd_int(l, n, g2, bound=1 << 10), 4)
    Ci = run(dd, Ai, Bi)
    assert np.array_equal(Ci[0], Ai[0] @ Bi[0])


@pytest.mark.parametrize("algo,lv", [("block", 0), ("strassen", 1), ("winograd", 2)])
def test_recursive_algorithms_with_ozaki_leaves(dd, algo, lv):
    g = inputs.rng(196)
    m, n, l = 130, 98, 140
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B, algo=algo, levels=lv)
    ii, jj = all_entries(m, n)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -200 * l


@pytest.mark.parametrize("n", [512, 1024])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1)])
def test_full_size_sampled_and_equal_accuracy_with_fma(dd, n, algo, lv):
    import torch
    g = inputs.rng(0)
    A = inputs.qd_uniform(n, n, g)
    B = inputs.qd_uniform(n, n, g)
    ii, jj = sample_entries(n, n, 120)
    Co = run(dd, A, B, algo=algo, levels=lv)
    Cf = to_host(dd.qd_gemm(to_dev(A), to_dev(B), algo=algo, levels=lv))
    torch.cuda.synchronize()
    eo = rownorm_error(A, B, Co, ii, jj)
    ef = rownorm_error(A, B, Cf, ii, jj)
    assert eo <= 2.0 ** -200 * n and ef <= 2.0 ** -200 * n, (eo, ef)
    assert eo <= 16 * ef + 2.0 ** -210, (eo, ef)


def test_row_scaled_variant(dd):
    n = 512
    g = inputs.rng(1)
    A = inputs.qd_uniform(n, n, g)
    B = inputs.qd_uniform(n, n, g)
    As, _ = inputs.row_scaled(A, g)
    ii, jj = sample_entries(n, n, 150)
    C = run(dd, As, B)
    assert rownorm_error(As, B, C, ii, jj) <= 2.0 ** -200 * n


def test_paper_matrices_closed_form(dd):
    import mpmath
    n = 1023
    A, B = inputs.paper_matrices(n, P=4)
    rows = list(range(0, n, 101)) + [n - 1]
    exact = inputs.paper_product_closed_form(n, rows)
    C = run(dd, A, B)
    with mpmath.workprec(400):
        worst = max(abs(sum(mpmath.mpf(float(C[c, r, j])) for c in range(4)) - ex) / ex
                    for r, ex in zip(rows, exact) for j in (0, n - 1))
    assert float(worst) <= 2.0 ** -200 * n


def test_zero_rows_and_columns(dd):
    g = inputs.rng(197)
    m, n, l = 40, 50, 60
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    A[:, 3, :] = 0.0
    B[:, :, 7] = 0.0
    C = run(dd, A, B)
    assert not C[:, 3, :].any() and not C[:, :, 7].any()
    ii, jj = all_entries(m, n)
    assert rownorm_error(A, B, C, ii, jj, den=np.maximum(rownorm_den(A, B), 1e-300)) <= \
        2.0 ** -200 * l


def test_deterministic(dd):
    g = inputs.rng(198)
    A = inputs.qd_uniform(150, 100, g)
    B = inputs.qd_uniform(100, 120, g)
    C1 = run(dd, A, B, algo="winograd", levels=1)
    C2 = run(dd, A, B, algo="winograd", levels=1)
    assert np.array_equal(C1, C2)
