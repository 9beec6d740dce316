"""Recorded call sequences (ddqd_graph_*): a replay equals the eager calls.

Each graph is replayed several times with other eager library work, torch
work and synchronisations in between; before every replay its outputs are
overwritten (NaN, or the original matrix for the in-place LU), and every
replay must reproduce the eager result bit for bit (same kernels, same
arguments).
"""
import numpy as np
import pytest

from paper_1510_08642_amd import inputs
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def _noise(dd, g):
    """Unrelated eager work between replays."""
    import torch
    X = to_dev(inputs.dd_uniform(70, 70, g))
    dd.dd_gemm(X, X, algo="winograd", levels=1)
    torch.cuda.synchronize()
    _ = (torch.randn(1000, device="cuda") * 2).sum().item()


@pytest.mark.parametrize("algo,levels,base,n", [("block", 0, "fma", 200), ("winograd", 1, "ozaki", 301),
                                                ("strassen", 2, "fma", 257), ("block", 0, "crt", 300),
                                                ("winograd", 1, "crt", 258)])
def test_gemm_replay_matches_eager(dd, algo, levels, base, n):
    import torch
    print(f"case graph gemm {algo}{levels} {base} n={n}", flush=True)
    g = inputs.rng(300 + n)
    A = to_dev(inputs.dd_uniform(n, n, g))
    B = to_dev(inputs.dd_uniform(n, n, g))
    ws = torch.empty(max(1, dd.gemm_workspace(2, n, n, n, algo, levels, base)), dtype=torch.uint8,
                     device="cuda")
    C_eager = dd.dd_gemm(A, B, algo=algo, levels=levels, base=base, ws=ws)
    torch.cuda.synchronize()
    ref = to_host(C_eager)
    C = torch.empty_like(C_eager)
    s = torch.cuda.Stream()
    graph = dd.capture(lambda: dd.dd_gemm(A, B, C, algo=algo, levels=levels, base=base, ws=ws), s)
    for rep in range(3):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay(s.cuda_stream)
        s.synchronize()
        assert np.array_equal(to_host(C), ref), rep
        _noise(dd, g)
    graph.release()


def test_lu_factor_and_solve_replay_matches_eager(dd):
    import torch
    n, nrhs = 300, 3
    print(f"case graph getrf+getrs n={n}", flush=True)
    g = inputs.rng(310)
    A0 = to_dev(inputs.dd_lu_matrix(n, g))
    B0 = to_dev(inputs.dd_uniform(n, nrhs, g))
    kw = dict(panel=64, algo="winograd", levels=1, base="ozaki")
    ws = torch.empty(max(1, dd.getrf_workspace(n, **kw)), dtype=torch.uint8, device="cuda")
    rws = torch.empty(max(1, dd.lib().dd_getrs_workspace(n, nrhs)), dtype=torch.uint8,
                      device="cuda")
    out = tuple(torch.empty(k, dtype=torch.int32, device="cuda") for k in (n, n, 1))
    A, B = A0.clone(), B0.clone()
    dd.dd_getrf(A, ws=ws, out=out, **kw)
    dd.dd_getrs(A, out[0], B, perm=out[1], ws=rws)
    torch.cuda.synchronize()
    ref = [to_host(A), to_host(B), to_host(out[0]), to_host(out[1])]

    def calls():
        dd.dd_getrf(A, ws=ws, out=out, **kw)
        dd.dd_getrs(A, out[0], B, perm=out[1], ws=rws)

    s = torch.cuda.Stream()
    graph = dd.capture(calls, s)
    for rep in range(3):
        A.copy_(A0)
        B.copy_(B0)
        out[0].fill_(-7)
        out[1].fill_(-7)
        torch.cuda.synchronize()
        graph.replay(s.cuda_stream)
        s.synchronize()
        got = [to_host(A), to_host(B), to_host(out[0]), to_host(out[1])]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        assert int(to_host(out[2])[0]) == 0
        _noise(dd, g)
    graph.release()


def test_grouped_replay_matches_eager(dd):
    import torch
    print("case graph grouped", flush=True)
    g = inputs.rng(320)
    shapes = [(64, 80, 96), (130, 70, 33), (200, 200, 200)]
    probs, refs = [], []
    for m, n, l in shapes:
        A = to_dev(inputs.dd_uniform(m, l, g))
        B = to_dev(inputs.dd_uniform(l, n, g))
        C = torch.empty((2, m, n), dtype=torch.float64, device="cuda")
        probs.append((A, B, C, 1, 0))
    dd.dd_gemm_grouped(probs)
    torch.cuda.synchronize()
    refs = [to_host(p[2]) for p in probs]
    s = torch.cuda.Stream()
    graph = dd.capture(lambda: dd.dd_gemm_grouped(probs, stream_of=s.cuda_stream), s)
    for rep in range(3):
        for p in probs:
            p[2].fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay(s.cuda_stream)
        s.synchronize()
        for p, r in zip(probs, refs):
            assert np.array_equal(to_host(p[2]), r), rep
        _noise(dd, g)
    graph.release()


def test_grouped_ozaki_replay_matches_eager(dd):
    """Grouped Ozaki products (exponents, slicing and products of several
    problems) recorded with their workspace and replayed: every replay gives
    the eager bits."""
    import torch
    print("case graph grouped ozaki", flush=True)
    g = inputs.rng(321)
    shapes = [(64, 80, 96), (130, 70, 33), (200, 200, 200), (1, 1, 1)]
    probs = []
    for m, n, l in shapes:
        A = to_dev(inputs.dd_uniform(m, l, g))
        B = to_dev(inputs.dd_uniform(l, n, g))
        C = torch.empty((2, m, n), dtype=torch.float64, device="cuda")
        probs.append((A, B, C, 1, 0, "ozaki", 0))
    ws = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")
    dd.dd_gemm_grouped(probs, ws=ws)
    torch.cuda.synchronize()
    refs = [to_host(p[2]) for p in probs]
    s = torch.cuda.Stream()
    graph = dd.capture(lambda: dd.dd_gemm_grouped(probs, ws=ws, stream_of=s.cuda_stream), s)
    for rep in range(3):
        for p in probs:
            p[2].fill_(float("nan"))
        ws.fill_(7)
        torch.cuda.synchronize()
        graph.replay(s.cuda_stream)
        s.synchronize()
        for p, r in zip(probs, refs):
            assert np.array_equal(to_host(p[2]), r), rep
        _noise(dd, g)
    graph.release()
