"""Pins of the LU comparison bounds (tests/lu_bounds.py) on the CPU: two of
the oracle's own unpivoted factorizations of the paper's Sec. 4 matrix, in
different rounding orders (blocked and unblocked), meet the backward-error
bound and agree within the first-order bound; a factor entry changed in its
last bits breaks the backward-error bound."""
import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.lu_bounds import da_bound, first_order_bound, split, vsum

UNIT = {2: 2.0 ** -100, 4: 2.0 ** -200}


def backward_error(A, LU):
    n = A.shape[1]
    L, U = split(LU)
    ii = np.repeat(np.arange(n), n)
    jj = np.tile(np.arange(n), n)
    back = np.abs(oracle.exact_entries(L, U, ii, jj, kout=1, alpha=-1, C0=A)[0]).reshape(n, n)
    return back, da_bound(L, U, UNIT[A.shape[0]])


@pytest.mark.parametrize("P,n", [(2, 96), (4, 48)])
def test_two_oracle_factorizations_meet_the_bounds(P, n):
    A = inputs.paper_random_matrix(n, inputs.rng(0), P)
    F1, p1, i1 = oracle.getrf(A, panel=32, pivot=False, algo="block", levels=0)
    F2, p2, i2 = oracle.getrf(A, panel=1, pivot=False, algo="block", levels=0)
    assert i1 == i2 == 0
    for F in (F1, F2):
        back, bound = backward_error(A, F)
        assert np.all(back <= bound)
    L1, U1 = split(F1)
    L2, U2 = split(F2)
    tol = 2 * (first_order_bound(L1, U1, da_bound(L1, U1, UNIT[P])) +
               first_order_bound(L2, U2, da_bound(L2, U2, UNIT[P])))
    assert np.all(np.abs(vsum(F1 - F2)) <= tol)


@pytest.mark.parametrize("P", [2, 4])
def test_a_wrong_factor_entry_breaks_the_backward_bound(P):
    n = 64
    A = inputs.paper_random_matrix(n, inputs.rng(1), P)
    F, _, _ = oracle.getrf(A, panel=16, pivot=False, algo="block", levels=0)
    for (i, j) in ((40, 7), (7, 40)):          # a multiplier, then an entry of U
        G = F.copy()
        G[P - 1, i, j] = G[P - 1, i, j] + np.ldexp(abs(G[0, i, j]), -70 if P == 2 else -160)
        back, bound = backward_error(A, G)
        assert np.any(back > bound), (i, j)
