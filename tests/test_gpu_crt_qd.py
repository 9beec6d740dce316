"""GPU parity of the CRT INT8-MFMA base in QD (qd_gemm base="crt").

Row i of A (scaled by 2^-e_i, max|a_ik| < 2^(e_i - 1)) and column j of B
(2^-f_j) are rounded to integers T of 214 bits, split T = H 2^108 + L
(|H| <= 2^106, |L| <= 2^107 (1 + 2^-35)); H_a H_b and the cross term
H_a L_b + L_a H_b are multiplied exactly by residues modulo N pairwise coprime
moduli, L_a L_b is dropped, and the rebuild runs in 270-bit (H H) and 162-bit
(cross) fixed point.  Bars, per entry against the exact product E (oracle):
    |C_ij - E_ij| <= l 2^(e_i + f_j - 215) (1 + 2^-30)       (roundings, L L)
                     + N 128 M (2^-484 + 2^-484) 2^(e_i + f_j)  (fixed point)
                     + 2^-198 (|E_ij| + l 2^(e_i + f_j - 215))   (QD arithmetic)
(the last from the worst-case bounds of the error-free summations into four
terms; far smaller in practice), the QD row-normwise tolerance 2^-200 l of
the other bases, and no more than 16 times the FMA base's error at full size.
Integer inputs need no rounding: the leading component of every entry is the
exact product when it fits one double.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import (all_entries, rownorm_den, rownorm_error, sample_entries, to_dev,
                           to_host, value_diff)

pytestmark = pytest.mark.gpu

TINY = 2.0 ** -1072


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def run(dd, A, B, C0=None, case="", **kw):
    import torch
    print(f"case qd crt {case} A={A.shape} B={B.shape} {kw}", flush=True)
    out = dd.qd_gemm(to_dev(A), to_dev(B), to_dev(C0) if C0 is not None else None, base="crt",
                     **kw)
    torch.cuda.synchronize()
    return to_host(out)


def scale_exp(x):
    mx = np.abs(x).max(axis=1)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + 1, 1)


def check_bound(dd, A, B, C, alpha=1, C0=None):
    """Every entry against the a-priori bound, on copies scaled by powers of
    two (row i by 2^s_i, column j by 2^t_j: each row and column maximum near
    1), where the oracle's exact products stay in the normal range; 2^(e_i +
    f_j) becomes 4 in those units."""
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
    ms = dd.crt_moduli(l, precision=4)
    M = math.prod(ms)
    kc = min(l, 32768)
    unit = 4.0  # 2^(e_i + f_j)
    rnd = l * unit * 2.0 ** -215 * (1 + 2.0 ** -30)
    chunks = -(-l // kc)
    fix = len(ms) * 128 * float(F(M, 2 ** 484) + F(M, 2 ** 484)) * unit * chunks
    arith = 2.0 ** -198 * (ex + rnd)
    tiny = np.ldexp(TINY, s[ii] + t[jj])
    bound = rnd + fix + arith + tiny
    if C0 is not None:  # the QD addition of C0
        bound = bound + 2.0 ** -200 * (ex + np.abs(C0s[0][ii, jj]))
    worst = float(np.max(err / bound))
    assert np.all(err <= bound), worst
    return worst


@pytest.mark.parametrize("shape", [(1, 1, 1), (32, 32, 32), (31, 33, 65), (70, 66, 75),
                                   (129, 97, 130), (3, 200, 97), (200, 1, 40), (257, 140, 96)])
def test_random_qd_vs_oracle_and_bound(dd, shape):
    m, n, l = shape
    g = inputs.rng(1180 + m + n)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B, case="random")
    ii, jj = all_entries(m, n)
    den = rownorm_den(A, B)
    e = rownorm_error(A, B, C, ii, jj, den=den)
    assert e <= 2.0 ** -200 * l, e
    check_bound(dd, A, B, C)
    Co = oracle.gemm(A, B, "block")
    d = float(np.max(value_diff(C, Co) / den[:, None]))
    assert d <= 2 * 2.0 ** -200 * l, d


@pytest.mark.parametrize("shape", [(9, 7, 11), (64, 64, 64), (130, 100, 257)])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1), ("strassen", 2)])
def test_integer_inputs(dd, shape, algo, lv):
    """Integers need no rounding and both integer products are exact; the
    rebuild leaves far below one unit of X_hh: the leading components
    are the exact product and the rest within the row-normwise tolerance."""
    m, n, l = shape
    g = inputs.rng(1170 + m)
    A = inputs.widen(inputs.dd_int(m, l, g), 4)
    B = inputs.widen(inputs.dd_int(l, n, g), 4)
    C = run(dd, A, B, case="integers", algo=algo, levels=lv)
    assert np.array_equal(C[0], A[0] @ B[0])
    den = rownorm_den(A, B)
    assert np.all(np.abs(C[1:]).sum(axis=0) <= 2.0 ** -200 * l * den[:, None])


def test_integers_beyond_two_doubles(dd):
    """70-bit integers: products of 140 bits, sums needing three doubles;
    both integer products are exact and the rebuild's fixed point leaves far
    below 2^-80 here, so what remains is the QD rounding of the rebuilt
    value, within 2^-205 of the exact integer."""
    g = np.random.default_rng(1171)
    m, n, l = 33, 40, 45
    Ai = [[int(g.integers(-(1 << 62), 1 << 62)) * 256 + int(g.integers(0, 256))
           for _ in range(l)] for _ in range(m)]
    Bi = [[int(g.integers(-(1 << 62), 1 << 62)) * 256 + int(g.integers(0, 256))
           for _ in range(n)] for _ in range(l)]

    def qd_from_ints(V):
        hi = np.array([[float(v) for v in row] for row in V])
        lo = np.array([[float(v - int(h)) for v, h in zip(row, hrow)]
                       for row, hrow in zip(V, hi)])
        z = np.zeros_like(hi)
        return np.stack([hi, lo, z, z])

    A, B = qd_from_ints(Ai), qd_from_ints(Bi)
    C = run(dd, A, B, case="70-bit integers")
    for i in range(0, m, 4):
        for j in range(0, n, 3):
            want = sum(Ai[i][k] * Bi[k][j] for k in range(l))
            got = sum(F(C[c, i, j]) for c in range(4))
            assert abs(got - want) <= abs(want) / 2 ** 205 + F(1, 2 ** 80), (i, j)


@pytest.mark.parametrize("alpha,beta", [(1, 1), (-1, 1), (-1, 0)])
def test_alpha_beta(dd, alpha, beta):
    g = inputs.rng(1190)
    m, n, l = 70, 45, 53
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C0 = inputs.qd_uniform(m, n, g)
    C = run(dd, A, B, C0=C0, case="alpha/beta", alpha=alpha, beta=beta)
    ii, jj = all_entries(m, n)
    e = rownorm_error(A, B, C, ii, jj, alpha=alpha, C0=C0 if beta else None)
    assert e <= 2.0 ** -200 * l, e
    check_bound(dd, A, B, C, alpha=alpha, C0=C0 if beta else None)


@pytest.mark.parametrize("algo,lv", [("winograd", 1), ("strassen", 2), ("winograd", 3)])
def test_recursive_forms_on_crt_leaves(dd, algo, lv):
    g = inputs.rng(1195 + lv)
    m, n, l = 300, 260, 280
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B, case="recursive", algo=algo, levels=lv)
    ii, jj = all_entries(m, n)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -200 * l


def test_long_k_uses_several_exact_chunks(dd):
    """l > 32768 (the cross product covers twice the chunk in one exact
    INT32 sum): two chunks, the second added to C in QD."""
    g = inputs.rng(1193)
    m, n, l = 24, 20, 33000
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    C = run(dd, A, B, case="long K")
    ii, jj = sample_entries(m, n, 24)
    assert rownorm_error(A, B, C, ii, jj) <= 2.0 ** -200 * l
    g2 = inputs.rng(1194)
    Ai = inputs.widen(inputs.dd_int(m, l, g2, bound=1 << 10), 4)
    Bi = inputs.widen(inputs.dd_int(l, n, g2, bound=1 << 10), 4)
    Ci = run(dd, Ai, Bi, case="long K integers")
    assert np.array_equal(Ci[0], Ai[0] @ Bi[0])


@pytest.mark.parametrize("n", [512, 1024])
@pytest.mark.parametrize("algo,lv", [("block", 0), ("winograd", 1)])
def test_full_size_sampled_and_equal_accuracy_with_fma(dd, n, algo, lv):
    import torch
    g = inputs.rng(0)
    A = inputs.qd_uniform(n, n, g)
    B = inputs.qd_uniform(n, n, g)
    ii, jj = sample_entries(n, n, 120)
    Cc = run(dd, A, B, case="full size", algo=algo, levels=lv)
    Cf = to_host(dd.qd_gemm(to_dev(A), to_dev(B), algo=algo, levels=lv))
    torch.cuda.synchronize()
    ec = rownorm_error(A, B, Cc, ii, jj)
    ef = rownorm_error(A, B, Cf, ii, jj)
    assert ec <= 2.0 ** -200 * n and ef <= 2.0 ** -200 * n, (ec, ef)
    assert ec <= 16 * ef + 2.0 ** -210, (ec, ef)


def test_row_scaled_variant(dd):
    n = 512
    g = inputs.rng(1)
    A = inputs.qd_uniform(n, n, g)
    B = inputs.qd_uniform(n, n, g)
    As, _ = inputs.row_scaled(A, g)
    ii, jj = sample_entries(n, n, 150)
    C = run(dd, As, B, case="row scaled")
    assert rownorm_error(As, B, C, ii, jj) <= 2.0 ** -200 * n


def test_deterministic(dd):
    g = inputs.rng(1198)
    A = inputs.qd_uniform(150, 100, g)
    B = inputs.qd_uniform(100, 120, g)
    C1 = run(dd, A, B, case="deterministic", algo="winograd", levels=1)
    C2 = run(dd, A, B, case="deterministic", algo="winograd", levels=1)
    assert np.array_equal(C1, C2)


# ---- the ends of the FP64 range ------------------------------------------------

def test_zero_rows_and_columns(dd):
    m, n, l = 130, 65, 200
    g = inputs.rng(1200)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    A[:, [0, 5, m - 1], :] = 0.0
    B[:, :, [1, n // 2, n - 1]] = 0.0
    B[:, :, 9] = 0.0
    B[:, 40, 9] = [0.75, 2.0 ** -60, 2.0 ** -115, 2.0 ** -170]
    C = run(dd, A, B, case="zero rows/columns")
    assert not C[:, [0, 5, m - 1], :].any()
    assert not C[:, :, [1, n // 2, n - 1]].any()
    check_bound(dd, A, B, C)


def test_subnormal_rows(dd):
    m, n, l = 64, 48, 96
    g = inputs.rng(1210)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    for r, e in ((3, -1040), (17, -1070)):
        A[0, r, :] = np.ldexp(A[0, r, :], e)
        A[1:, r, :] = 0.0
    C = run(dd, A, B, case="subnormal rows")
    check_bound(dd, A, B, C)
    assert np.any(C[0, 3] != 0.0)


@pytest.mark.parametrize("exp", [1000, -900])
def test_rows_near_the_range_ends(dd, exp):
    m, n, l = 96, 70, 130
    g = inputs.rng(1220)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    r = g.integers(exp - 8, exp + 1 if exp > 0 else exp + 8, m)
    A = np.ldexp(A, r[None, :, None])
    C = run(dd, A, B, case=f"rows near 2^{exp}")
    check_bound(dd, A, B, C)


def test_wide_spread_inside_rows(dd):
    m, n, l = 64, 64, 160
    g = inputs.rng(1240)
    A = inputs.qd_uniform(m, l, g)
    B = inputs.qd_uniform(l, n, g)
    A = np.ldexp(A, g.integers(-100, 101, (m, l))[None])
    B = np.ldexp(B, g.integers(-100, 101, (l, n))[None])
    C = run(dd, A, B, case="spread 2^+-100")
    check_bound(dd, A, B, C)


# ---- LU with CRT trailing updates -----------------------------------------------

@pytest.mark.parametrize("n,panel", [(300, 64), (1024, 128)])
def test_qd_lu_with_crt_updates(dd, n, panel):
    """QD factorization with trailing updates on the CRT base (partial
    pivoting): the solve's residual, formed exactly by the oracle on sampled
    rows, within n 2^-200 of ||A|| ||x||."""
    import torch
    print(f"case qd crt lu n={n} panel={panel}", flush=True)
    g = inputs.rng(1250 + n)
    A = inputs.qd_lu_matrix(n, g, boost=False)
    LU = to_dev(A)
    ipiv, perm, info = dd.qd_getrf(LU, panel=panel, algo="winograd", levels=1, base="crt")
    b = inputs.qd_uniform(n, 1, g)
    X = to_dev(b)
    dd.qd_getrs(LU, ipiv, X, perm=perm)
    torch.cuda.synchronize()
    assert int(to_host(info)[0]) == 0
    x = to_host(X)
    rows = np.arange(0, n, 7 if n < 500 else 37)
    r = oracle.exact_entries(A[:, rows, :], x, np.arange(len(rows)),
                             np.zeros(len(rows), dtype=np.int64), kout=1, alpha=-1,
                             C0=b[:, rows, :])[0]
    normA = np.max(np.sum(np.abs(A[0]), axis=1))
    assert np.max(np.abs(r)) / (normA * np.max(np.abs(x[0]))) <= n * 2.0 ** -200
