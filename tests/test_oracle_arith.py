"""Pins for the oracle's arithmetic against exact rational arithmetic.

Every check here compares the oracle with ``fractions.Fraction`` (exact
rationals), never with the oracle itself: the error-free transformations
must be exact, expansions must carry exactly the sum of their inputs, and
DD / QD operations must stay inside the published relative error bounds
(DD add about 3u^2, DD mul below 5u^2, u = 2^-53; QD about 2^-208).
"""
from fractions import Fraction as F

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_1510_08642_amd import inputs

U = 2.0 ** -53

moderate = st.floats(min_value=-1e100, max_value=1e100, allow_nan=False,
                     allow_infinity=False).filter(lambda x: x == 0.0 or abs(x) > 1e-100)


def fr(v):
    return sum((F(float(x)) for x in np.ravel(v)), F(0))


@settings(max_examples=300, deadline=None)
@given(moderate, moderate)
def test_two_sum_exact(a, b):
    s, e = oracle.eft("two_sum", [a], [b])
    assert F(s[0]) + F(e[0]) == F(a) + F(b)
    assert s[0] == a + b


@settings(max_examples=300, deadline=None)
@given(moderate, moderate)
def test_fast_two_sum_exact_when_ordered(a, b):
    if abs(a) < abs(b):
        a, b = b, a
    s, e = oracle.eft("fast_two_sum", [a], [b])
    assert F(s[0]) + F(e[0]) == F(a) + F(b)


@settings(max_examples=300, deadline=None)
@given(st.floats(min_value=-1e80, max_value=1e80, allow_nan=False).filter(
    lambda x: x == 0.0 or abs(x) > 1e-80),
       st.floats(min_value=-1e80, max_value=1e80, allow_nan=False).filter(
    lambda x: x == 0.0 or abs(x) > 1e-80))
def test_two_prod_exact(a, b):
    p, e = oracle.eft("two_prod", [a], [b])
    assert F(p[0]) + F(e[0]) == F(a) * F(b)
    assert p[0] == a * b


def _lowbit(x: float) -> F:
    """Value of the lowest set bit of a nonzero double."""
    p, q = abs(float(x)).as_integer_ratio()
    if q > 1:
        return F(1, q)
    return F(p & -p)


def _nonoverlapping_increasing(e):
    for lo, hi in zip(e[:-1], e[1:]):
        assert abs(lo) < abs(hi)
        # every bit of lo lies below the lowest set bit of hi
        assert F(abs(float(lo))) < _lowbit(hi)


@settings(max_examples=100, deadline=None)
@given(st.lists(moderate, min_size=1, max_size=40))
def test_expansion_sum_is_exact_and_nonoverlapping(vals):
    e = oracle.expansion_sum(vals)
    assert fr(e) == sum((F(v) for v in vals), F(0))
    _nonoverlapping_increasing(list(e))


@settings(max_examples=100, deadline=None)
@given(st.lists(moderate, min_size=1, max_size=40))
def test_expansion_round_leading_terms(vals):
    exact = sum((F(v) for v in vals), F(0))
    r = oracle.expansion_round(vals, 4)
    if exact == 0:
        assert np.all(r == 0)
        return
    # four leading terms carry about 4*52 bits
    assert abs(fr(r) - exact) <= abs(exact) * F(2) ** -205


def _dd_batch(n, g, scale=1.0):
    X = inputs.dd_uniform(1, n, g)
    return np.ascontiguousarray(np.stack([X[0, 0] * scale, X[1, 0] * scale], axis=1))


def _qd_batch(n, g):
    X = inputs.qd_uniform(1, n, g)
    return np.ascontiguousarray(np.stack([X[c, 0] for c in range(4)], axis=1))


@pytest.mark.parametrize("seed", [0, 1])
def test_dd_ops_error_bounds(seed):
    g = inputs.rng(seed)
    x = _dd_batch(400, g)
    y = _dd_batch(400, g)
    # include cancellation-heavy pairs: y close to -x
    y[:50] = -x[:50]
    y[:50, 1] = y[:50, 1] * 0.5
    for op, bound in [("add", 3 * U * U * (1 + 8 * U)), ("sub", 3 * U * U * (1 + 8 * U)),
                      ("mul", 5 * U * U), ("div", 6 * U * U)]:
        z = oracle.elementwise(op, x, y)
        worst = 0.0
        for t in range(len(x)):
            a, b = fr(x[t]), fr(y[t])
            ex = {"add": a + b, "sub": a - b, "mul": a * b, "div": a / b}[op]
            got = fr(z[t])
            if ex == 0:
                assert got == 0
                continue
            rel = abs(got - ex) / abs(ex)
            worst = max(worst, float(rel))
            # result is a normalised DD: |lo| <= ulp(hi)/2
            assert z[t, 0] + z[t, 1] == z[t, 0]
        assert worst <= bound, (op, worst / (U * U))


@pytest.mark.parametrize("seed", [0, 1])
def test_qd_ops_error_bounds(seed):
    g = inputs.rng(seed)
    x = _qd_batch(200, g)
    y = _qd_batch(200, g)
    y[:30] = -x[:30]
    y[:30, 3] *= 0.25
    for op in ["add", "sub", "mul", "div"]:
        z = oracle.elementwise(op, x, y)
        for t in range(len(x)):
            a, b = fr(x[t]), fr(y[t])
            ex = {"add": a + b, "sub": a - b, "mul": a * b, "div": a / b}[op]
            got = fr(z[t])
            if ex == 0:
                assert got == 0
                continue
            assert abs(got - ex) <= abs(ex) * F(2) ** -205, op


def test_exact_dot_expansion_equals_fraction_sum():
    g = inputs.rng(3)
    for P, gen in [(2, inputs.dd_uniform), (4, inputs.qd_uniform)]:
        x = gen(1, 37, g)[:, 0, :]
        y = gen(1, 37, g)[:, 0, :]
        y[:, 5] = -y[:, 5]
        e = oracle.exact_dot_expansion(x, y)
        want = sum(fr(x[:, k]) * fr(y[:, k]) for k in range(37))
        assert fr(e) == want


def test_exact_entries_against_fraction():
    g = inputs.rng(4)
    A = inputs.dd_uniform(5, 9, g)
    B = inputs.dd_uniform(9, 4, g)
    C0 = inputs.dd_uniform(5, 4, g)
    ii = np.repeat(np.arange(5), 4)
    jj = np.tile(np.arange(4), 5)
    for alpha, c0 in [(1, None), (-1, C0)]:
        out = oracle.exact_entries(A, B, ii, jj, kout=4, alpha=alpha, C0=c0)
        err = oracle.exact_error(A, B, out[:2], ii, jj, alpha=alpha, C0=c0)
        for t, (i, j) in enumerate(zip(ii, jj)):
            ex = alpha * sum(fr(A[:, i, k]) * fr(B[:, k, j]) for k in range(9))
            if c0 is not None:
                ex += fr(c0[:, i, j])
            assert abs(fr(out[:, t]) - ex) <= abs(ex) * F(2) ** -205
            # the error routine returns (exact - computed DD), rounded once
            d = ex - fr(out[:2, t])
            assert abs(F(err[t]) - d) <= abs(d) * F(2) ** -51


def test_mpmath_cross_check_dd_and_qd():
    """Independent check with mpmath at 700 bits on sampled entries."""
    import mpmath
    g = inputs.rng(5)
    for P, gen in [(2, inputs.dd_uniform), (4, inputs.qd_uniform)]:
        A = gen(6, 50, g)
        B = gen(50, 6, g)
        ii, jj = np.array([0, 3, 5]), np.array([1, 4, 0])
        out = oracle.exact_entries(A, B, ii, jj, kout=4)
        with mpmath.workprec(700):
            for t, (i, j) in enumerate(zip(ii, jj)):
                ex = mpmath.fsum(mpmath.fsum(mpmath.mpf(float(c)) for c in A[:, i, k]) *
                                 mpmath.fsum(mpmath.mpf(float(c)) for c in B[:, k, j])
                                 for k in range(50))
                got = mpmath.fsum(mpmath.mpf(float(c)) for c in out[:, t])
                assert abs(got - ex) <= abs(ex) * mpmath.mpf(2) ** -205
