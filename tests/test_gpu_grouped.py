"""GPU parity of dd_gemm_grouped: uneven problems in one persistent launch.

Each problem's result must be bit-identical to the same product launched on
its own (dd_gemm, Block, FMA base) and within the DD tolerance of the exact
product; a problem's bits must not depend on the other members of the group.
"""
import numpy as np
import pytest

from paper_1510_08642_amd import inputs
from tests.helpers import all_entries, rownorm_error, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


SHAPES = [(64, 64, 64), (1, 1, 1), (130, 7, 65), (7, 200, 3), (100, 100, 0), (0, 5, 5),
          (257, 129, 300), (33, 1, 90), (64, 65, 1), (500, 40, 77)]


def make(g, shapes):
    out = []
    for (m, n, l) in shapes:
        A = inputs.dd_uniform(m, l, g)
        B = inputs.dd_uniform(l, n, g)
        C0 = inputs.dd_uniform(m, n, g)
        out.append((A, B, C0))
    return out


def test_grouped_bitwise_equal_to_single_calls(dd):
    import torch
    g = inputs.rng(300)
    probs = make(g, SHAPES)
    singles, group = [], []
    for k, (A, B, C0) in enumerate(probs):
        alpha, beta = (1, 0) if k % 3 == 0 else ((-1, 1) if k % 3 == 1 else (1, 1))
        Cs = to_dev(C0)
        dd.dd_gemm(to_dev(A), to_dev(B), Cs, alpha=alpha, beta=beta, algo="block")
        singles.append(Cs)
        group.append((to_dev(A), to_dev(B), to_dev(C0), alpha, beta))
    print("case grouped", len(group), flush=True)
    dd.dd_gemm_grouped(group)
    torch.cuda.synchronize()
    for k, ((A, B, C0), s, gp) in enumerate(zip(probs, singles, group)):
        assert np.array_equal(to_host(s), to_host(gp[2])), k
        alpha, beta = gp[3], gp[4]
        m, n = A.shape[1], B.shape[2]
        if m and n and A.shape[2]:
            ii, jj = all_entries(m, n)
            e = rownorm_error(A, B, to_host(gp[2]), ii, jj, alpha=alpha,
                              C0=C0 if beta else None)
            assert e <= 2.0 ** -100 * A.shape[2], (k, e)


def test_group_membership_does_not_change_results(dd):
    import torch
    g = inputs.rng(301)
    probs = make(g, SHAPES[:6] * 5)          # 30 problems: two launches of <= 24
    full = [(to_dev(A), to_dev(B), to_dev(C0), 1, 0) for (A, B, C0) in probs]
    dd.dd_gemm_grouped(full)
    alone = [(to_dev(A), to_dev(B), to_dev(C0), 1, 0) for (A, B, C0) in probs[:3]]
    dd.dd_gemm_grouped(alone)
    torch.cuda.synchronize()
    for a, f in zip(alone, full[:3]):
        assert np.array_equal(to_host(a[2]), to_host(f[2]))


def test_grouped_alias_rejected(dd):
    g = inputs.rng(302)
    A = to_dev(inputs.dd_uniform(8, 8, g))
    B = to_dev(inputs.dd_uniform(8, 8, g))
    C = to_dev(inputs.dd_uniform(8, 8, g))
    with pytest.raises(dd.DDQDError):
        dd.dd_gemm_grouped([(A, B, C, 1, 0), (C, B, A, 1, 0)])
    with pytest.raises(dd.DDQDError):
        dd.dd_gemm_grouped([(A, B, C, 1, 0), (A, B, C, 1, 0)])


# ---- Ozaki leaves in grouped launches ---------------------------------------

@pytest.mark.parametrize("slices", [0, 12])
def test_grouped_ozaki_bitwise_equal_to_single_calls(dd, slices):
    """Ozaki problems of mixed shapes (more than one group of 12), every
    alpha / beta form, each bit-identical to its own dd_gemm call with the
    Ozaki base, and within the DD tolerance (S = 16) of the exact product."""
    import torch
    g = inputs.rng(310 + slices)
    shapes = SHAPES + [(300, 260, 513), (64, 128, 1000), (95, 33, 64), (2, 300, 40),
                       (128, 128, 128)]
    probs = make(g, shapes)
    singles, group = [], []
    for k, (A, B, C0) in enumerate(probs):
        alpha, beta = (1, 0) if k % 3 == 0 else ((-1, 1) if k % 3 == 1 else (1, 1))
        Cs = to_dev(C0)
        dd.dd_gemm(to_dev(A), to_dev(B), Cs, alpha=alpha, beta=beta, algo="block",
                   base="ozaki", slices=slices)
        singles.append(Cs)
        group.append((to_dev(A), to_dev(B), to_dev(C0), alpha, beta))
    print(f"case grouped ozaki {len(group)} problems slices={slices}", flush=True)
    dd.dd_gemm_grouped(group, base="ozaki", slices=slices)
    torch.cuda.synchronize()
    for k, ((A, B, C0), s, gp) in enumerate(zip(probs, singles, group)):
        assert np.array_equal(to_host(s), to_host(gp[2])), (k, shapes[k])
        m, n, l = A.shape[1], B.shape[2], A.shape[2]
        if m and n and l and slices == 0:
            ii, jj = all_entries(m, n)
            e = rownorm_error(A, B, to_host(gp[2]), ii, jj, alpha=gp[3],
                              C0=C0 if gp[4] else None)
            assert e <= 2.0 ** -100 * l, (k, e)


def test_grouped_mixed_bases_slices_and_long_k(dd):
    """FMA and Ozaki problems, two slice counts and one problem whose K needs
    two exact chunks (l > 16384, run on its own) in one call: every result
    bit-identical to its own call."""
    import torch
    g = inputs.rng(320)
    cases = [((70, 80, 90), "fma", 0), ((70, 80, 90), "ozaki", 0), ((33, 64, 100), "ozaki", 14),
             ((40, 36, 17000), "ozaki", 0), ((128, 64, 64), "ozaki", 14), ((5, 5, 5), "fma", 0),
             ((200, 100, 64), "ozaki", 0)]
    group, singles = [], []
    for (m, n, l), base, S in cases:
        A, B = inputs.dd_uniform(m, l, g), inputs.dd_uniform(l, n, g)
        Ad, Bd = to_dev(A), to_dev(B)
        singles.append(dd.dd_gemm(Ad, Bd, algo="block", base=base, slices=S))
        C = torch.empty((2, m, n), dtype=torch.float64, device=Ad.device)
        group.append((Ad, Bd, C, 1, 0, base, S))
    print("case grouped mixed bases", flush=True)
    dd.dd_gemm_grouped(group)
    torch.cuda.synchronize()
    for k, (s, gp) in enumerate(zip(singles, group)):
        assert torch.equal(s, gp[2]), (k, cases[k])


def test_grouped_ozaki_membership_and_repeat(dd):
    """A problem's bits do not depend on the other members of its group, and
    a repeated call reproduces them."""
    import torch
    g = inputs.rng(330)
    probs = make(g, [(100, 90, 80), (64, 64, 64), (150, 20, 300), (1, 1, 1), (77, 130, 65)] * 3)
    full = [(to_dev(A), to_dev(B), to_dev(C0), 1, 1) for (A, B, C0) in probs]
    dd.dd_gemm_grouped(full, base="ozaki")
    alone = [(to_dev(A), to_dev(B), to_dev(C0), 1, 1) for (A, B, C0) in probs[2:4]]
    dd.dd_gemm_grouped(alone, base="ozaki")
    again = [(to_dev(A), to_dev(B), to_dev(C0), 1, 1) for (A, B, C0) in probs]
    dd.dd_gemm_grouped(again, base="ozaki")
    torch.cuda.synchronize()
    for a, f in zip(alone, full[2:4]):
        assert torch.equal(a[2], f[2])
    for a, f in zip(again, full):
        assert torch.equal(a[2], f[2])
