"""Autotuner (dd_gemm_tune / qd_gemm_tune, algo="auto"; the paper's Sec. 5
open parameters: block size and recursion depth per shape).

The tuned configuration must be a correct product: algo="auto" reproduces
the explicit call with the chosen algorithm and depth bit for bit (the
Block tile does not change any entry's operation order), and its error
against the oracle's exact products stays within the DD/QD bound.
"""
import numpy as np
import pytest

from paper_1510_08642_amd import inputs
from tests.helpers import rownorm_error, sample_entries, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    ddqd.tune_clear()
    return ddqd


def _err_ok(A, B, C, P, l):
    ii, jj = sample_entries(A.shape[1], B.shape[2], 64)
    bound = (2.0 ** -100 if P == 2 else 2.0 ** -200) * l
    return rownorm_error(A, B, C, ii, jj) <= bound


@pytest.mark.parametrize("P,m,n,l,base", [(2, 70, 75, 66, "fma"), (2, 256, 256, 256, "fma"),
                                          (2, 300, 200, 310, "ozaki"), (2, 300, 200, 310, "crt"),
                                          (4, 130, 130, 130, "fma"), (4, 300, 200, 310, "crt")])
def test_tuned_choice_is_cached_and_exact_to_the_explicit_call(dd, P, m, n, l, base):
    import torch
    print(f"case tune P={P} {m}x{n}x{l} {base}", flush=True)
    g = inputs.rng(400 + m)
    mk = inputs.dd_uniform if P == 2 else inputs.qd_uniform
    A, B = mk(m, l, g), mk(l, n, g)
    Ad, Bd = to_dev(A), to_dev(B)
    r = dd.tune(Ad, Bd, base=base, reps=2)
    assert r["candidates"] >= 2 and r["ms"] > 0
    assert dd.tune_lookup(P, m, n, l, base=base) == r
    gem = dd.dd_gemm if P == 2 else dd.qd_gemm
    kw = dict(base=base)
    Ca = to_host(gem(Ad, Bd, algo="auto", **kw))
    Ce = to_host(gem(Ad, Bd, algo=r["algo"], levels=r["levels"], **kw))
    torch.cuda.synchronize()
    assert np.array_equal(Ca, Ce)
    assert _err_ok(A, B, Ca, P, l)


def test_default_small_tile_is_bit_identical_to_64(dd):
    import torch
    dd.tune_clear()
    g = inputs.rng(410)
    A, B = inputs.dd_uniform(100, 90, g), inputs.dd_uniform(90, 110, g)
    Ad, Bd = to_dev(A), to_dev(B)
    assert dd.tune_lookup(2, 100, 110, 90)["tile"] == 32
    Ca = to_host(dd.dd_gemm(Ad, Bd, algo="auto"))          # Block, 32 x 32 tiles
    Cb = to_host(dd.dd_gemm(Ad, Bd, algo="block"))         # Block, 64 x 64 tiles
    torch.cuda.synchronize()
    assert np.array_equal(Ca, Cb)
    C0 = to_dev(inputs.dd_uniform(100, 110, g))
    Cc = to_host(dd.dd_gemm(Ad, Bd, C0.clone(), alpha=-1, beta=1, algo="auto"))
    Cd = to_host(dd.dd_gemm(Ad, Bd, C0.clone(), alpha=-1, beta=1, algo="block"))
    assert np.array_equal(Cc, Cd)


def test_qd_small_tile_is_bit_identical_to_32(dd):
    """The QD Block kernel's 16x16 tile (the default for small products)
    gives the 32x32 tile's bits, with and without beta."""
    import torch
    dd.tune_clear()
    g = inputs.rng(411)
    A, B = inputs.qd_uniform(100, 90, g), inputs.qd_uniform(90, 110, g)
    Ad, Bd = to_dev(A), to_dev(B)
    assert dd.tune_lookup(4, 100, 110, 90)["tile"] == 16
    Ca = to_host(dd.qd_gemm(Ad, Bd, algo="auto"))
    Cb = to_host(dd.qd_gemm(Ad, Bd, algo="block"))
    torch.cuda.synchronize()
    assert np.array_equal(Ca, Cb)
    assert _err_ok(A, B, Ca, 4, 90)
    C0 = to_dev(inputs.qd_uniform(100, 110, g))
    Cc = to_host(dd.qd_gemm(Ad, Bd, C0.clone(), alpha=-1, beta=1, algo="auto"))
    Cd = to_host(dd.qd_gemm(Ad, Bd, C0.clone(), alpha=-1, beta=1, algo="block"))
    assert np.array_equal(Cc, Cd)


@pytest.mark.parametrize("P", [2, 4])
def test_tuned_ozaki_band_is_bit_identical(dd, P):
    """Ozaki leaves: the tuner times tile orders in bands of 2..16 tile rows;
    the chosen order gives the default order's bits."""
    import torch
    print(f"case tune ozaki band P={P}", flush=True)
    dd.tune_clear()
    g = inputs.rng(412 + P)
    mk = inputs.dd_uniform if P == 2 else inputs.qd_uniform
    m, n, l = 520, 390, 300
    Ad, Bd = to_dev(mk(m, l, g)), to_dev(mk(l, n, g))
    r = dd.tune(Ad, Bd, base="ozaki", reps=2)
    assert r["candidates"] >= 4
    gem = dd.dd_gemm if P == 2 else dd.qd_gemm
    Ca = gem(Ad, Bd, algo="auto", base="ozaki")
    Ce = gem(Ad, Bd, algo=r["algo"], levels=r["levels"], base="ozaki")
    torch.cuda.synchronize()
    assert torch.equal(Ca, Ce), r


@pytest.mark.parametrize("P,n,base", [(2, 300, "ozaki"), (2, 70, "fma"), (4, 200, "fma")])
def test_lu_panel_tuner_picks_a_width_and_auto_reproduces_it(dd, P, n, base):
    """ddqd_getrf_tune times the panel widths K = 32 alpha <= n (Sec. 4's
    sweep) on a copy of A; panel="auto" then factors with the chosen width,
    bit for bit as the explicit call, and A is left unchanged."""
    import torch
    print(f"case lu panel tune P={P} n={n} {base}", flush=True)
    dd.tune_clear()
    g = inputs.rng(420 + n)
    A = (inputs.dd_lu_matrix if P == 2 else inputs.qd_lu_matrix)(n, g)
    Ad = to_dev(A)
    kw = dict(algo="winograd", levels=1, base=base)
    r = dd.getrf_tune(Ad, reps=1, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(Ad), A)
    widths = [32 * a for a in range(1, 11) if 32 * a <= n]
    assert r["panel"] in widths and r["candidates"] == len(widths) and r["ms"] > 0
    assert dd.getrf_panel_lookup(P, n, **kw) == r
    getrf = dd.dd_getrf if P == 2 else dd.qd_getrf
    A1, A2 = Ad.clone(), Ad.clone()
    f1 = getrf(A1, panel="auto", **kw)
    f2 = getrf(A2, panel=r["panel"], **kw)
    torch.cuda.synchronize()
    assert torch.equal(A1, A2)
    assert torch.equal(f1[0], f2[0]) and torch.equal(f1[1], f2[1])
    assert int(to_host(f1[2])[0]) == 0
    # an order whose width was not tuned keeps the default
    assert dd.getrf_panel_lookup(P, n + 1, **kw)["panel"] == 128


@pytest.mark.parametrize("P", [2, 4])
def test_crt_256_tiles_give_the_128_tiles_bits(dd, P):
    """With K below two leaves' minimum the CRT candidates are the two Block
    tiles only, timed 128 x 128 first; C then holds the 256 x 256 tiles'
    product (each wave 4 x 4 MFMA blocks, two K blocks a barrier), which must
    equal the default 128 x 128 call bit for bit: the tile changes only the
    order of exact integer sums."""
    import torch
    print(f"case tune crt tiles P={P}", flush=True)
    g = inputs.rng(430 + P)
    mk = inputs.dd_uniform if P == 2 else inputs.qd_uniform
    m, n, l = 300, 270, 20
    A, B = mk(m, l, g), mk(l, n, g)
    Ad, Bd = to_dev(A), to_dev(B)
    C256 = torch.empty((P, m, n), dtype=torch.float64, device=Ad.device)
    r = dd.tune(Ad, Bd, C256, base="crt", reps=1)
    assert r["candidates"] == 2
    gem = dd.dd_gemm if P == 2 else dd.qd_gemm
    C128 = gem(Ad, Bd, algo="block", base="crt")
    torch.cuda.synchronize()
    C256h, C128h = to_host(C256), to_host(C128)
    assert np.array_equal(C256h, C128h)
    assert _err_ok(A, B, C128h, P, l)
