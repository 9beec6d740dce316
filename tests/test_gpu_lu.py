"""GPU parity of dd_getrf / dd_getrs (Sec. 4, steps 1-3 and Eq. 2).

Checked against the oracle and against structure:
  * pivots: the interchange sequence equals the oracle's (partial pivoting
    decided in DD) on random matrices, and the permutation vector equals the
    interchanges replayed on the identity;
  * factors: elementwise against the oracle's blocked LU within
    n 2^-96 max|LU| (both are DD computations that differ in rounding order);
  * exact cases: diagonal / upper triangular / integer L U / permutation;
  * solve: residual ||b - A x||_inf / (||A||_inf ||x||_inf) <= n 2^-100,
    formed exactly by the oracle; the paper's x = [0, 1, ..., n-1] is
    recovered with a forward error within ||A^-1|| times the exactly formed
    residual (plus b's rounding), and within the solves' first-order
    backward-error bound of the oracle's solve on the same factors.
"""
import numpy as np
import pytest

import oracle
from tests import lu_bounds
from paper_1510_08642_amd import inputs
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def factor(dd, A, **kw):
    import torch
    print(f"case getrf n={A.shape[1]} {kw}", flush=True)
    Ad = to_dev(A)
    ipiv, perm, info = dd.dd_getrf(Ad, **kw)
    torch.cuda.synchronize()
    return to_host(Ad), to_host(ipiv), (to_host(perm) if perm is not None else None), \
        int(to_host(info)[0])


def solve(dd, LU, ipiv, B, perm=None):
    import torch
    Bd = to_dev(B)
    dd.dd_getrs(to_dev(LU), to_dev(ipiv), Bd, perm=to_dev(perm) if perm is not None else None)
    torch.cuda.synchronize()
    return to_host(Bd)


def ddm(hi):
    hi = np.asarray(hi, dtype=np.float64)
    return np.stack([hi, np.zeros_like(hi)])


@pytest.mark.parametrize("n,panel", [(1, 4), (7, 4), (37, 16), (64, 32), (100, 24), (150, 64),
                                     (257, 128)])
@pytest.mark.parametrize("algo,levels", [("block", 0), ("winograd", 1)])
def test_random_vs_oracle(dd, n, panel, algo, levels):
    g = inputs.rng(200 + n)
    A = inputs.dd_lu_matrix(n, g, boost=False)
    LU, ipiv, perm, info = factor(dd, A, panel=panel, algo=algo, levels=levels)
    LUo, ipo, info_o = oracle.getrf(A, panel=panel, pivot=True, algo=algo, levels=levels)
    assert info == info_o == 0
    assert np.array_equal(ipiv, ipo)
    rows = list(range(n))
    for i, p in enumerate(ipiv):
        rows[i], rows[p] = rows[p], rows[i]
    assert np.array_equal(perm, rows)
    scale = np.max(np.abs(LUo[0]))
    diff = np.abs((LU[0] - LUo[0]) + (LU[1] - LUo[1]))
    assert np.max(diff) <= n * 2.0 ** -96 * scale


@pytest.mark.parametrize("pivot", ["none", "partial"])
def test_structured_exact(dd, pivot):
    g = inputs.rng(210)
    n = 45
    D = np.diag(g.uniform(1, 2, n))
    LU, ipiv, _, info = factor(dd, ddm(D), panel=16, pivot=pivot)
    assert info == 0 and np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(LU[0], D) and not LU[1].any()
    Up = np.triu(g.uniform(-1, 1, (n, n))) + np.diag(np.full(n, 4.0))
    LU, ipiv, _, info = factor(dd, ddm(Up), panel=16, pivot=pivot, algo="strassen", levels=1)
    assert np.array_equal(LU[0], Up) and not LU[1].any()


@pytest.mark.parametrize("algo,levels,base", [("block", 0, "fma"), ("winograd", 2, "fma"),
                                              ("winograd", 1, "ozaki")])
def test_integer_factors_recovered_exactly(dd, algo, levels, base):
    g = inputs.rng(211)
    n = 70
    L = np.tril(g.integers(-3, 4, (n, n)), -1) + np.eye(n, dtype=np.int64)
    d = 2.0 ** g.integers(-2, 3, n)
    U = np.triu(g.integers(-3, 4, (n, n)), 1).astype(np.float64) + np.diag(d)
    A = L.astype(np.float64) @ U
    LU, ipiv, _, info = factor(dd, ddm(A), panel=32, pivot="none", algo=algo, levels=levels,
                               base=base)
    assert info == 0
    assert np.array_equal(np.tril(LU[0], -1), np.tril(L, -1).astype(np.float64))
    assert np.array_equal(np.triu(LU[0]), U)
    assert not LU[1].any()


def test_permutation_and_singular(dd):
    n = 23
    g = inputs.rng(212)
    perm = g.permutation(n)
    Pm = np.zeros((n, n))
    Pm[np.arange(n), perm] = 1.0
    LU, ipiv, pv, info = factor(dd, ddm(Pm), panel=8)
    assert info == 0
    assert np.array_equal(Pm[pv], np.eye(n))
    assert np.array_equal(LU[0], np.eye(n))
    S = np.ones((12, 12))
    S[0, 0] = 2.0
    _, _, _, info = factor(dd, ddm(S), panel=4)
    assert info == 3                  # same as the oracle's pin


@pytest.mark.parametrize("n,nrhs,use_perm", [(50, 1, True), (130, 3, False), (200, 16, True),
                                             (97, 20, True)])
def test_solve_residual_and_paper_solution(dd, n, nrhs, use_perm):
    g = inputs.rng(220 + n)
    A = inputs.dd_lu_matrix(n, g, boost=False)
    LU, ipiv, perm, _ = factor(dd, A, panel=32)
    B = inputs.dd_uniform(n, nrhs, g)
    X = solve(dd, LU, ipiv, B, perm if use_perm else None)
    assert oracle.lu_residual(A, X, B) <= n * 2.0 ** -100
    # the paper's test solution x = [0, 1, ..., n-1], b := A x formed exactly
    # and rounded to DD
    x = ddm(np.arange(n, dtype=np.float64)[:, None])
    b = oracle.exact_entries(A, x, np.arange(n), np.zeros(n, dtype=np.int64), kout=2)
    b = b.reshape(2, n, 1)
    xs = solve(dd, LU, ipiv, b, perm if use_perm else None)

    def fwd(X):
        return np.max(np.abs((X[0, :, 0] - np.arange(n)) + X[1, :, 0]))
    # the whole path: x_hat - x = A^-1 (A x_hat - b) + A^-1 (b - A x), the
    # residual formed exactly and b's rounding to DD below 2^-104 |b|; the
    # inverse is taken in FP64 (a factor 2 covers its relative error)
    r = oracle.exact_entries(A, xs, np.arange(n), np.zeros(n, dtype=np.int64), kout=1,
                             alpha=-1, C0=b)[0]
    normAinv = np.max(np.sum(np.abs(np.linalg.inv(A[0])), axis=1))
    bound = 2 * normAinv * (np.max(np.abs(r)) + 2.0 ** -104 * np.max(np.abs(b[0])))
    assert fwd(xs) <= bound, (fwd(xs), bound)
    # the two triangular solves alone: the oracle's DD solve on the GPU's own
    # factors (same factors, different rounding order in the solves) differs
    # from the GPU's by at most the first-order effect of both solves'
    # backward errors (the GPU's applies computed inverses of its 64-row
    # diagonal blocks)
    xg = oracle.getrs(LU, ipiv, b)
    diff = np.abs((xs[0] - xg[0]) + (xs[1] - xg[1]))[:, 0]
    assert np.all(diff <= lu_bounds.solve_diff_bound(LU, xg, 2.0 ** -104, block=64)[:, 0])


def test_solution_matches_oracle_solve(dd):
    g = inputs.rng(230)
    n = 120
    A = inputs.dd_lu_matrix(n, g, boost=False)
    B = inputs.dd_uniform(n, 4, g)
    LU, ipiv, perm, _ = factor(dd, A, panel=32, algo="winograd", levels=1)
    X = solve(dd, LU, ipiv, B, perm)
    LUo, ipo, _ = oracle.getrf(A, panel=32, pivot=True, algo="winograd", levels=1)
    Xo = oracle.getrs(LUo, ipo, B)
    scale = np.max(np.abs(Xo[0]))
    assert np.max(np.abs((X[0] - Xo[0]) + (X[1] - Xo[1]))) <= n * 2.0 ** -94 * scale


@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("panel,algo,levels,base", [(64, "winograd", 1, "fma"),
                                                    (128, "winograd", 2, "ozaki"),
                                                    (256, "block", 0, "ozaki")])
def test_config3_full_size_residual(dd, n, panel, algo, levels, base):
    g = inputs.rng(0)
    A = inputs.dd_lu_matrix(n, g)
    b = inputs.dd_uniform(n, 1, g)
    LU, ipiv, perm, info = factor(dd, A, panel=panel, algo=algo, levels=levels, base=base)
    assert info == 0
    x = solve(dd, LU, ipiv, b, perm)
    # sampled exact residual rows (the full one is n^2 exact products)
    rows = np.unique(np.concatenate([np.arange(0, n, max(1, n // 200)), [n - 1]]))
    r = oracle.exact_entries(A[:, rows, :], x, np.arange(len(rows)),
                             np.zeros(len(rows), dtype=np.int64), kout=1, alpha=-1,
                             C0=b[:, rows, :])[0]
    normA = np.max(np.sum(np.abs(A[0]), axis=1))
    res = np.max(np.abs(r)) / (normA * np.max(np.abs(x[0])))
    assert res <= n * 2.0 ** -100, res


def test_winograd_update_error_close_to_block(dd):
    """Sec. 4: no visible error increase from the Winograd update on a random
    matrix; here within a factor of 16 of the Block update's residual."""
    g = inputs.rng(240)
    n = 300
    A = inputs.dd_lu_matrix(n, g, boost=False)
    B = inputs.dd_uniform(n, 1, g)
    res = {}
    for algo, lv in [("block", 0), ("winograd", 3)]:
        LU, ipiv, perm, _ = factor(dd, A, panel=64, algo=algo, levels=lv)
        res[algo] = oracle.lu_residual(A, solve(dd, LU, ipiv, B, perm), B)
    assert res["winograd"] <= 16 * res["block"] + n * 2.0 ** -106


@pytest.mark.parametrize("n,panel,vals", [(100, 32, (-1, 1)), (129, 64, (-2, -1, 0, 1, 2)),
                                          (300, 128, (-1, 1))])
def test_pivot_ties_pick_first_row(dd, n, panel, vals):
    """Integer matrices: exact ties in |a_ic| are frequent; partial pivoting
    takes the first maximal row, as the oracle does (Sec. 4 with pivoting)."""
    g = inputs.rng(250 + n)
    A = ddm(g.choice(np.array(vals, dtype=np.float64), size=(n, n)))
    LU, ipiv, _, info = factor(dd, A, panel=panel)
    LUo, ipo, info_o = oracle.getrf(A, panel=panel, pivot=True, algo="block", levels=0)
    assert info == info_o
    assert np.array_equal(ipiv, ipo)
    if info == 0:
        scale = np.max(np.abs(LUo[0]))
        assert np.max(np.abs((LU[0] - LUo[0]) + (LU[1] - LUo[1]))) <= n * 2.0 ** -96 * scale


def test_pivot_decided_by_low_words(dd):
    """Candidates with equal high words: the low words decide (DD compare)."""
    n = 40
    g = inputs.rng(260)
    A = inputs.dd_lu_matrix(n, g, boost=False)
    A[:, :, 0] = 0.0
    A[0, [3, 11, 17, 30], 0] = [1.0, 1.0, -1.0, 0.5]
    A[1, [3, 11, 17, 30], 0] = [2.0 ** -60, 2.0 ** -58, -(2.0 ** -57), 2.0 ** -55]
    LU, ipiv, _, info = factor(dd, A, panel=16)
    LUo, ipo, _ = oracle.getrf(A, panel=16, pivot=True, algo="block", levels=0)
    assert ipiv[0] == ipo[0] == 17
    assert np.array_equal(ipiv, ipo)


# ---- the paper's row-wise parallel comparator (panel width 0) --------------

@pytest.mark.parametrize("n", [1, 2, 7, 100, 300])
def test_rowwise_vs_oracle_unblocked(dd, n):
    """Row-wise elimination without pivoting is the unblocked right-looking LU:
    the oracle's blocked LU with panel width 1 and no pivoting."""
    g = inputs.rng(240 + n)
    A = inputs.dd_lu_matrix(n, g)
    LU, ipiv, perm, info = factor(dd, A, panel=0, pivot="none")
    LUo, ipo, info_o = oracle.getrf(A, panel=1, pivot=False, algo="block", levels=0)
    assert info == info_o == 0
    assert np.array_equal(ipiv, np.arange(n)) and np.array_equal(perm, np.arange(n))
    assert np.max(np.abs((LU[0] - LUo[0]) + (LU[1] - LUo[1]))) <= \
        n * 2.0 ** -96 * np.max(np.abs(LUo[0]))
    b = inputs.dd_uniform(n, 2, g)
    x = solve(dd, LU, ipiv, b, perm)
    assert oracle.lu_residual(A, x, b) <= n * 2.0 ** -100


def test_rowwise_integer_factors_exact(dd):
    g = inputs.rng(250)
    n = 60
    L = np.tril(g.integers(-3, 4, (n, n)), -1) + np.eye(n, dtype=np.int64)
    d = 2.0 ** g.integers(-2, 3, n)
    U = np.triu(g.integers(-3, 4, (n, n)), 1).astype(np.float64) + np.diag(d)
    A = np.stack([L.astype(np.float64) @ U, np.zeros((n, n))])
    LU, _, _, info = factor(dd, A, panel=0, pivot="none")
    assert info == 0
    assert np.array_equal(np.tril(LU[0], -1), np.tril(L, -1).astype(np.float64))
    assert np.array_equal(np.triu(LU[0]), U)
    assert not LU[1].any()


def test_rowwise_zero_pivots_set_info(dd):
    """An exactly zero pivot: info = its 1-based column, the step is skipped
    (as the blocked form does); the last pivot is checked too."""
    n = 5
    A = np.stack([np.eye(n), np.zeros((n, n))])
    A[0, 2, 2] = 0.0
    _, _, _, info = factor(dd, A, panel=0, pivot="none")
    assert info == 3
    A = np.stack([np.eye(n), np.zeros((n, n))])
    A[0, n - 1, n - 1] = 0.0
    _, _, _, info = factor(dd, A, panel=0, pivot="none")
    assert info == n


@pytest.mark.parametrize("P", [2, 4])
def test_getrs_with_the_device_busy_is_bit_identical(dd, P):
    """A block step of the solve is one launch whose workgroups all read the
    diagonal block as it is in memory; while a large product keeps the device
    busy on another stream, workgroups of the step start late, and the solve
    must still give the result of the quiet device, bit for bit.  The same for
    the factorisation (whose panel steps also read, in one launch, values
    that later launches overwrite)."""
    import torch
    print(f"case getrs busy P={P}", flush=True)
    n, nrhs = 300, 3
    g = inputs.rng(21)
    gen = inputs.dd_lu_matrix if P == 2 else inputs.qd_lu_matrix
    LU = to_dev(gen(n, g))
    getrf = dd.dd_getrf if P == 2 else dd.qd_getrf
    getrs = dd.dd_getrs if P == 2 else dd.qd_getrs
    A0 = LU.clone()
    ipiv, perm, info = getrf(LU, panel=64)
    B = to_dev((inputs.dd_uniform if P == 2 else inputs.qd_uniform)(n, nrhs, g))
    ref = B.clone()
    getrs(LU, ipiv, ref, perm=perm)
    torch.cuda.synchronize()
    m = 2048
    A2 = to_dev(inputs.dd_uniform(m, m, g))
    B2 = to_dev(inputs.dd_uniform(m, m, g))
    C2 = torch.empty_like(A2)
    ws2 = torch.empty(dd.gemm_workspace(2, m, m, m, "block", 0, "ozaki"), dtype=torch.uint8,
                      device=A2.device)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(6):
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s1):
            for _ in range(2):
                dd.dd_gemm(A2, B2, C2, base="ozaki", ws=ws2)
        with torch.cuda.stream(s2):
            X = B.clone()
            getrs(LU, ipiv, X, perm=perm)
            LU2 = A0.clone()
            ipiv2, _, _ = getrf(LU2, panel=64)
        torch.cuda.synchronize()
        assert torch.equal(X, ref), rep
        assert torch.equal(LU2, LU) and torch.equal(ipiv2, ipiv), rep


def test_latency_probe_runs(dd):
    """The diagnostic behind the strip kernel's profile: every chain reports a
    positive latency, and a TwoSum (dependent adds) takes longer than one add."""
    for threads in (64, 1024):
        r = dd.latency_probe(threads, steps=256)
        assert all(v > 0 for v in r.values()), r
        assert r["two_sum"] > r["add"]
