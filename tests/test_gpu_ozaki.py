"""GPU parity of the Ozaki INT8-MFMA base (dd_gemm base="ozaki").

Bars: integer inputs bit-exact (all digits fit in the slices, every dropped
diagonal is zero); random DD within the row-normwise tolerance 2^-100 l and,
per entry, within the method's a-priori bound
    |C_ij - E_ij| <= l (S + 3) 2^(-7S - 2) 2^(e_i + f_j) + 2^-104 |E_ij|
(e_i, f_j the scaling exponents: max|a_ik| < 2^(e_i - 1)); and agreement with
the FMA base at equal accuracy.
"""
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
    print(f"case ozaki A={A.shape} B={B.shape} {kw}", flush=True)
    out = dd.dd_gemm(to_dev(A), to_dev(B), to_dev(C0) if C0 is not None else None, **kw)
    torch.cuda.synchronize()
    return to_host(out)


def scale_exp(x):
    """e with max|x| < 2^(e-1), per row, from the leading components."""
    mx = np.abs(x).max(axis=1)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + 1, 1)


def apriori_ok(A, B, C, ii, jj, S, alpha=1, C0=None):
    l = A.shape[2]
    err = np.abs(oracle.exact_error(A, B, C, ii, jj, alpha=alpha, C0=C0))
    ea = scale_exp(A[0])
    fb = scale_exp(B[0].T)
    ex = np.abs(oracle.exact_entries(A, B, ii, jj, kout=1, alpha=alpha, C0=C0)[0])
    bound = l * (S + 3) * np.ldexp(1.0, -7 * S - 2 + ea[ii] + fb[jj]) + 2.0 ** -104 * ex
    return bool(np.all(err <= bound)), float(np.max(err / bound))


@pytest.mark.parametrize("shape", [(9, 7, 11), (64, 64, 64), (65, 66, 67), (130, 100, 257)])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1), ("strassen", 2)])
def test_integer_inputs_bit_exact(dd, shape, algo, lv):
    m, n, l = shape
    g = inputs.rng(70 + m)
    A = inputs.dd_int(m, l, g)
    B = inputs.dd_int(l, n, g)
    C = run(dd, A, B, algo=algo, levels=lv, base="ozaki")
    assert np.array_equal(C[0], A[0] @ B[0])
    assert not C[1].any()


@pytest.mark.parametrize("shape", [(1, 1, 1), (32, 32, 32), (63, 65, 67), (128, 128, 128),
                                   (129, 130, 131), (200, 1, 77), (3, 300, 500)])
def test_random_dd_vs_oracle_and_bound(dd, shape):
    m, n, l = shape
    g = inputs.rng(80 + m + n)
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, base="ozaki")
    ii, jj = all_entries(m, n)
    den = rownorm_den(A, B)
    e = rownorm_error(A, B, C, ii, jj, den=den)
    assert e <= 2.0 ** -100 * l, e
    ok, worst = apriori_ok(A, B, C, ii, jj, 16)
    assert ok, worst
    Co = oracle.gemm(A, B, "block")
    d = float(np.max(value_diff(C, Co) / den[:, None]))
    assert d <= 2 * 2.0 ** -100 * l, d


@pytest.mark.parametrize("alpha,beta", [(1, 1), (-1, 1), (-1, 0)])
def test_alpha_beta(dd, alpha, beta):
    g = inputs.rng(90)
    m, n, l = 70, 45, 53
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C0 = inputs.dd_uniform(m, n, g)
    C = run(dd, A, B, C0=C0, alpha=alpha, beta=beta, base="ozaki")
    ii, jj = all_entries(m, n)
    e = rownorm_error(A, B, C, ii, jj, alpha=alpha, C0=C0 if beta else None)
    assert e <= 2.0 ** -100 * l, e


@pytest.mark.parametrize("S", [8, 10, 12, 14, 15, 16, 17, 18, 20])
def test_slice_count_meets_apriori_bound(dd, S):
    g = inputs.rng(91)
    m, n, l = 96, 80, 150
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, base="ozaki", slices=S)
    ii, jj = all_entries(m, n)
    ok, worst = apriori_ok(A, B, C, ii, jj, S)
    assert ok, (S, worst)


def test_more_slices_is_more_accurate(dd):
    g = inputs.rng(92)
    m, n, l = 64, 64, 256
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    ii, jj = all_entries(m, n)
    errs = [rownorm_error(A, B, run(dd, A, B, base="ozaki", slices=S), ii, jj)
            for S in (8, 10, 12, 14)]
    assert all(errs[i + 1] < errs[i] / 1000 for i in range(len(errs) - 1)), errs


def test_long_k_uses_several_exact_chunks(dd):
    """l > 16384 K values per exact INT32 accumulation: two chunks."""
    g = inputs.rng(93)
    m, n, l = 40, 36, 20000
    A = inputs.dd_uniform(m, l, g)
    B = inputs.dd_uniform(l, n, g)
    C = run(dd, A, B, base="ozaki")
    ii, jj = sample_entries(m, n, 60)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -100 * l
    # integer inputs through the chunked path stay exact
    g2 = inputs.rng(94)
    Ai, Bi = inputs.dd_int(m, l, g2, bound=1 << 10), inputs.dd_int(l, n, g2, bound=1 << 10)
    Ci = run(dd, Ai, Bi, base="ozaki")
    assert np.array_equal(Ci[0], Ai[0] @ Bi[0])


def test_row_scaled_variant_and_equal_accuracy_with_fma(dd):
    n = 1024
    g = inputs.rng(1)
    A = inputs.dd_uniform(n, n, g)
    B = inputs.dd_uniform(n, n, g)
    As, _ = inputs.row_scaled(A, g)
    ii, jj = sample_entries(n, n, 300)
    for X in (A, As):
        Co = run(dd, X, B, base="ozaki")
        Cf = run(dd, X, B, base="fma")
        eo = rownorm_error(X, B, Co, ii, jj)
        ef = rownorm_error(X, B, Cf, ii, jj)
        assert eo <= 2.0 ** -100 * n and ef <= 2.0 ** -100 * n
        # equal accuracy: the Ozaki error is within a small factor of the FMA one
        assert eo <= 16 * ef + 2.0 ** -104, (eo, ef)


@pytest.mark.parametrize("n", [1024, 2048])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1), ("winograd", 2),
                                     ("strassen", 3)])
def test_config1_full_size_sampled(dd, n, algo, lv):
    g = inputs.rng(0)
    A = inputs.dd_uniform(n, n, g)
    B = inputs.dd_uniform(n, n, g)
    C = run(dd, A, B, algo=algo, levels=lv, base="ozaki")
    ii, jj = sample_entries(n, n, 200)
    e = rownorm_error(A, B, C, ii, jj)
    assert e <= 2.0 ** -100 * n, e


def test_paper_matrices_closed_form(dd):
    import mpmath
    n = 1025
    A, B = inputs.paper_matrices(n)
    rows = list(range(0, n, 101)) + [n - 1]
    exact = inputs.paper_product_closed_form(n, rows)
    C = run(dd, A, B, base="ozaki")
    with mpmath.workprec(300):
        worst = max(abs(mpmath.mpf(float(C[0, r, j])) + mpmath.mpf(float(C[1, r, j])) - ex) / ex
                    for r, ex in zip(rows, exact) for j in (0, n - 1))
    assert float(worst) <= 2.0 ** -100 * n


def test_deterministic(dd):
    g = inputs.rng(95)
    A = inputs.dd_uniform(300, 200, g)
    B = inputs.dd_uniform(200, 250, g)
    C1 = run(dd, A, B, base="ozaki", algo="winograd", levels=1)
    C2 = run(dd, A, B, base="ozaki", algo="winograd", levels=1)
    assert np.array_equal(C1, C2)
