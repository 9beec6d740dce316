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
                                          (2, 300, 200, 310, "ozaki"), (4, 130, 130, 130, "fma")])
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
    kw = dict(base=base) if P == 2 else {}
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
