"""GPU parity of the paper's own LU experiment (Sec. 4, Fig. 5): the random
matrix with entries in [-1, 1], no pivoting, block size K = alpha n_min
(n_min = 32), trailing updates by Block or Winograd (FMA leaves) and by Block
on Ozaki leaves, in DD and QD, against the oracle's blocked LU without
pivoting.

Without pivoting this matrix has small pivots and large multipliers (growth
of about 10^4 at n = 1024), so two correct factorizations in different
rounding orders differ far above n u |LU|.  The bars are therefore the ones
elimination itself guarantees:
  * backward error of the factors, formed exactly on sampled entries:
    |A - L U|_ij <= n u max((|L||U|)_ij, max_k |l_ik| max_k |u_kj|)
    (u = 2^-100 DD, 2^-200 QD; the second term is the row / column form of
    the Ozaki leaves' bound);
  * elementwise agreement with the oracle's factors within twice the
    first-order perturbation bound of the LU factorization: for dA bounded
    as above, X = |L^-1| dA |U^-1| bounds L^-1 dL + dU U^-1, so
    |dU| <= triu(X) |U| and |dL| <= |L| tril(X, -1) for each factorization,
    and the two differ by at most the sum (a factor 2 more for the
    first-order truncation);
  * the solve of the paper's x = [0, 1, ..., n-1]: residual
    |b - A x|_i <= 3 n u (dA-bound |x|)_i on sampled rows (backward
    stability of the two triangular solves), and the forward error within
    ||A^-1|| ||A x - b|| (x - x* = A^-1 (A x - b), the residual formed
    exactly);
  * no interchanges (ipiv = perm = identity) and info = 0, as the oracle.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import to_dev, to_host
from tests.lu_bounds import da_bound, first_order_bound, samples, split, vsum

pytestmark = pytest.mark.gpu

UNIT = {2: 2.0 ** -100, 4: 2.0 ** -200}


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


@functools.lru_cache(maxsize=None)
def paper_matrix(n, P):
    return inputs.paper_random_matrix(n, inputs.rng(0), P)


@functools.lru_cache(maxsize=None)
def oracle_factors(n, P):
    LU, ipiv, info = oracle.getrf(paper_matrix(n, P), panel=64, pivot=False, algo="block",
                                  levels=0)
    return LU, ipiv, info


def run(dd, P, n, K, algo, levels, base):
    import torch
    print(f"case paper lu P={P} n={n} K={K} {algo}{levels} {base}", flush=True)
    A = paper_matrix(n, P)
    Ad = to_dev(A)
    getrf = dd.dd_getrf if P == 2 else dd.qd_getrf
    ipiv, perm, info = getrf(Ad, panel=K, pivot="none", algo=algo, levels=levels, base=base)
    torch.cuda.synchronize()
    return A, Ad, to_host(Ad), to_host(ipiv), to_host(perm), int(to_host(info)[0])


def check_factorization(P, A, LU, ipiv, perm, info, compare_oracle):
    n = A.shape[1]
    u = UNIT[P]
    assert info == 0
    assert np.array_equal(ipiv, np.arange(n)) and np.array_equal(perm, np.arange(n))
    L, U = split(LU)
    dA = da_bound(L, U, u)
    ii, jj = samples(n, 600, n + P)
    back = np.abs(oracle.exact_entries(L, U, ii, jj, kout=1, alpha=-1, C0=A)[0])
    assert np.all(back <= dA[ii, jj]), float(np.max(back / dA[ii, jj]))
    if compare_oracle:
        LUo, ipo, info_o = oracle_factors(n, P)
        assert info_o == 0 and np.array_equal(ipo, np.arange(n))
        Lo, Uo = split(LUo)
        tol = 2 * (first_order_bound(L, U, dA) + first_order_bound(Lo, Uo, da_bound(Lo, Uo, u)))
        diff = np.abs(vsum(LU - LUo))
        assert np.all(diff <= tol), float(np.max(diff / tol))
    return L, U, dA


def check_paper_solution(dd, P, A, Ad, L, U, dA):
    """x = [0, ..., n-1], b = A x formed exactly; the library's solve."""
    import torch
    n = A.shape[1]
    x = np.zeros((P, n, 1))
    x[0, :, 0] = np.arange(n)
    b = oracle.exact_entries(A, x, np.arange(n), np.zeros(n, dtype=np.int64), kout=P)
    b = b.reshape(P, n, 1)
    X = to_dev(b)
    getrs = dd.dd_getrs if P == 2 else dd.qd_getrs
    getrs(Ad, torch.from_numpy(np.arange(n, dtype=np.int32)).to(Ad.device), X)
    torch.cuda.synchronize()
    xs = to_host(X)
    r = oracle.exact_entries(A, xs, np.arange(n), np.zeros(n, dtype=np.int64), kout=1, alpha=-1,
                             C0=b)[0]
    ax = np.abs(xs[0, :, 0])
    assert np.all(np.abs(r) <= 3 * (dA @ ax) + 2.0 ** -1000), \
        float(np.max(np.abs(r) / (3 * (dA @ ax))))
    # x - [0..n-1] = A^-1 r + A^-1 (b - A [0..n-1]), the second term from b's
    # rounding to P terms (relative error below 2^-104 / 2^-208); the inverse
    # is taken in FP64 (a factor 2 covers its error)
    fwd = np.max(np.abs(vsum(xs[:, 1:, 0]) - np.arange(1, n)))
    normAinv = np.max(np.sum(np.abs(np.linalg.inv(A[0])), axis=1))
    b_round = (2.0 ** -104 if P == 2 else 2.0 ** -208) * np.max(np.abs(b[0]))
    assert fwd <= 2 * normAinv * (np.max(np.abs(r)) + b_round), fwd
    rel = float(np.max(np.abs(vsum(xs[:, 1:, 0]) - np.arange(1, n)) / np.arange(1, n)))
    print(f"  max relative error of x: {rel:.3e}", flush=True)


UPDATES = [("block", "fma"), ("winograd", "fma"), ("block", "ozaki")]


def levels_for(algo, K):
    # the paper's Winograd update recurses down to n_min = 32: alpha = K / 32
    return 0 if algo == "block" else max(1, (K // 32).bit_length() - 1)


@pytest.mark.parametrize("n,K", [(256, 32), (256, 96), (256, 160), (256, 320), (512, 64),
                                 (512, 192), (512, 320), (1024, 32), (1024, 128),
                                 (1024, 320)])
@pytest.mark.parametrize("algo,base", UPDATES)
def test_dd_paper_lu(dd, n, K, algo, base):
    lv = levels_for(algo, K)
    A, Ad, LU, ipiv, perm, info = run(dd, 2, n, K, algo, lv, base)
    L, U, dA = check_factorization(2, A, LU, ipiv, perm, info, compare_oracle=True)
    check_paper_solution(dd, 2, A, Ad, L, U, dA)


@pytest.mark.parametrize("n,K,oracle_cmp", [(256, 32, True), (256, 96, True), (256, 160, True),
                                            (512, 64, False), (512, 320, False)])
@pytest.mark.parametrize("algo,base", UPDATES)
def test_qd_paper_lu(dd, n, K, oracle_cmp, algo, base):
    lv = levels_for(algo, K)
    A, Ad, LU, ipiv, perm, info = run(dd, 4, n, K, algo, lv, base)
    L, U, dA = check_factorization(4, A, LU, ipiv, perm, info, compare_oracle=oracle_cmp)
    check_paper_solution(dd, 4, A, Ad, L, U, dA)


@pytest.mark.parametrize("P", [2, 4])
def test_rowwise_comparator_on_the_paper_matrix(dd, P):
    """The paper's row-wise parallel LU (panel width 0) on the same matrix."""
    n = 256
    A, Ad, LU, ipiv, perm, info = run(dd, P, n, 0, "block", 0, "fma")
    L, U, dA = check_factorization(P, A, LU, ipiv, perm, info, compare_oracle=True)
    check_paper_solution(dd, P, A, Ad, L, U, dA)
