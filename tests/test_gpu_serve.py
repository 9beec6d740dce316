"""Serving on the GPU: a mixed stream of DD products and LU solves with
Poisson arrivals runs through the continuous-batching loop; every result is
bit-identical to the same request run alone (no batching, one slot), and
sampled results meet the DD tolerance against the exact answer."""
import numpy as np
import pytest

import oracle
from paper_1510_08642_amd import inputs
from tests.helpers import sample_entries, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import serve
    pools = serve.DevicePools(nmax_gemm=512, nmax_lu=512, nrhs_max=16, seed=0)
    return serve, pools


def build(serve, pools, seed, count=60, rate=3000.0):
    trace = inputs.serving_trace(count, rate=rate, seed=seed, gemm_n=(32, 512), lu_n=(64, 512),
                                 nrhs=(1, 16))
    reqs = serve.make_requests(trace)
    for r in reqs:
        r.payload = pools.payload(r)
    return reqs


@pytest.mark.parametrize("base", ["fma", "ozaki"])
def test_mixed_stream_equals_alone(env, base):
    import torch
    serve, pools = env
    print(f"case serve base={base}", flush=True)
    mix = build(serve, pools, seed=11)
    ex = serve.GpuExecutor(slots=4, base=base, gemm_algo="winograd", gemm_levels=1)
    st = serve.Server(ex, budget_bytes=1 << 30, slots=4, small_n=256).run(mix)
    assert st.completed == len(mix) and st.failed == 0
    assert st.batches < len(mix)              # some products were grouped (either base)
    alone = build(serve, pools, seed=11)
    for k, r in enumerate(alone):
        r.t_arrive = 0.0
    ex1 = serve.GpuExecutor(slots=1, base=base, gemm_algo="winograd", gemm_levels=1)
    for r in alone:
        serve.Server(ex1, budget_bytes=1 << 30, slots=1, small_n=0).run([r])
    torch.cuda.synchronize()
    for a, b in zip(mix, alone):
        assert np.array_equal(to_host(a.result), to_host(b.result)), (a.rid, a.kind, a.n)


def test_sampled_results_within_tolerance(env):
    serve, pools = env
    reqs = build(serve, pools, seed=12, count=30)
    ex = serve.GpuExecutor(slots=3, base="fma")
    serve.Server(ex, budget_bytes=1 << 30, slots=3).run(reqs)
    checked = 0
    for r in reqs:
        A, B = (to_host(x.contiguous()) for x in r.payload)
        R = to_host(r.result)
        if r.kind == "gemm":
            ii, jj = sample_entries(r.n, r.n, 20, seed=r.rid)
            err = np.abs(oracle.exact_error(A, B, R, ii, jj))
            den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)[ii]
            assert np.max(err / den) <= 2.0 ** -100 * r.n
        else:
            assert oracle.lu_residual(A, R, B) <= r.n * 2.0 ** -100
        checked += 1
    assert checked == 30


def test_resident_factorization(env):
    serve, pools = env
    ex = serve.GpuExecutor(slots=1, base="fma")
    A = pools.la[:, :300, :300]
    key = ex.factorize(A, "k")
    for seed in range(3):
        B = pools.lb[:, :300, seed:seed + 2]
        X = ex.solve(key, B)
        assert oracle.lu_residual(to_host(A.contiguous()), to_host(X),
                                  to_host(B.contiguous())) <= 300 * 2.0 ** -100
    ex.release(key)
    assert "k" not in ex.factors


def test_online_server_matches_direct_calls(env):
    """Live submissions from two threads while earlier ones run; every
    future's result is bit-identical to the same library calls made alone."""
    import threading

    import torch
    serve, pools = env
    from paper_1510_08642_amd import ddqd as dd
    print("case online server", flush=True)
    reqs = build(serve, pools, seed=13, count=40)
    ex = serve.GpuExecutor(slots=3, base="fma", gemm_algo="winograd", gemm_levels=1)
    srv = serve.OnlineServer(ex, budget_bytes=1 << 30, slots=3, small_n=256)
    futs = [None] * len(reqs)

    def submit(ks):
        for k in ks:
            A, B = reqs[k].payload
            futs[k] = srv.submit_gemm(A, B) if reqs[k].kind == "gemm" else \
                srv.submit_lu_solve(A, B)
    th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    got = [f.result(timeout=120) for f in futs]
    srv.close(timeout=120)
    torch.cuda.synchronize()
    assert srv.stats().completed == len(reqs)
    for r, x in zip(reqs, got):
        A, B = r.payload
        if r.kind == "gemm":
            small = r.n <= 256
            ref = dd.dd_gemm(A, B, algo="block" if small else "winograd", levels=0 if small else 1)
        else:
            LU = A.clone()
            ipiv, perm, _ = dd.dd_getrf(LU, panel=min(128, r.n), algo="winograd", levels=1)
            ref = B.clone()
            dd.dd_getrs(LU, ipiv, ref, perm=perm)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(x), to_host(ref)), (r.rid, r.kind, r.n)


# ---- the serving workload at its full sizes --------------------------------

@pytest.fixture(scope="module")
def full_pools():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import serve
    return serve.DevicePools(nmax_gemm=1024, nmax_lu=2048, nrhs_max=16, seed=0)


def check_result(r):
    """A product on sampled entries against the exact product (row-normwise
    <= 2^-100 n); a solve by its residual on sampled rows, formed exactly
    (||b - A x||_inf / (||A||_inf ||x||_inf) <= n 2^-100)."""
    A, B = (to_host(x.contiguous()) for x in r.payload)
    R = to_host(r.result)
    if r.kind == "gemm":
        ii, jj = sample_entries(r.n, r.n, 24, seed=r.rid)
        err = np.abs(oracle.exact_error(A, B, R, ii, jj))
        den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)[ii]
        e = float(np.max(err / den))
        assert e <= 2.0 ** -100 * r.n, (r.rid, r.n, e)
        return e
    n, nrhs = r.n, r.nrhs
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(r.rid).integers(0, n, 40)]))
    ii = np.repeat(np.arange(len(rows)), nrhs)
    jj = np.tile(np.arange(nrhs), len(rows))
    res = oracle.exact_entries(A[:, rows, :], R, ii, jj, kout=1, alpha=-1, C0=B[:, rows, :])[0]
    normA = np.max(np.sum(np.abs(A[0]), axis=1))
    e = float(np.max(np.abs(res)) / (normA * np.max(np.abs(R[0]))))
    assert e <= n * 2.0 ** -100, (r.rid, n, nrhs, e)
    return e


@pytest.mark.parametrize("base", ["fma", "ozaki"])
def test_config4_full_size_every_result_checked(full_pools, base):
    """240 requests of the serving workload (60 % products with n
    log-uniform in [64, 1024], 40 % LU factor-and-solve with n in
    [128, 2048] and 1-16 right-hand sides), Poisson arrivals, four slots:
    every result is checked."""
    import torch

    from paper_1510_08642_amd import serve
    print(f"case serve full size base={base}", flush=True)
    trace = inputs.serving_trace(240, rate=2000.0, seed=21)
    reqs = serve.make_requests(trace)
    for r in reqs:
        r.payload = full_pools.payload(r)
    assert max(r.n for r in reqs if r.kind == "gemm") > 900
    assert max(r.n for r in reqs if r.kind == "lu") > 1500
    ex = serve.GpuExecutor(slots=4, base=base)
    st = serve.Server(ex, budget_bytes=1 << 30, slots=4).run(reqs)
    torch.cuda.synchronize()
    assert st.completed == len(reqs) and st.failed == 0
    worst = {"gemm": 0.0, "lu": 0.0}
    for r in reqs:
        worst[r.kind] = max(worst[r.kind], check_result(r))
    print(f"  worst product error {worst['gemm']:.3e}, worst residual {worst['lu']:.3e}, "
          f"batches {st.batches}", flush=True)


@pytest.mark.parametrize("base", ["fma", "ozaki"])
def test_full_size_mix_equals_alone(full_pools, base):
    """30 requests including the largest product (n = 1024) and the largest
    solve (n = 2048, 16 right-hand sides): each result in the mix is
    bit-identical to the same request run alone."""
    import torch

    from paper_1510_08642_amd import serve
    print(f"case serve full-size mix vs alone base={base}", flush=True)

    def make():
        trace = inputs.serving_trace(28, rate=2000.0, seed=22)
        t_mid = trace[len(trace) // 2]["t_arrive"]
        trace.insert(3, dict(kind="gemm", n=1024, nrhs=0, t_arrive=trace[3]["t_arrive"], seed=0))
        trace.insert(15, dict(kind="lu", n=2048, nrhs=16, t_arrive=t_mid, seed=0))
        reqs = serve.make_requests(trace)
        for r in reqs:
            r.payload = full_pools.payload(r)
        return reqs
    mix = make()
    ex = serve.GpuExecutor(slots=4, base=base)
    st = serve.Server(ex, budget_bytes=1 << 30, slots=4).run(mix)
    assert st.completed == len(mix) == 30
    alone = make()
    ex1 = serve.GpuExecutor(slots=1, base=base)
    for r in alone:
        r.t_arrive = 0.0
        serve.Server(ex1, budget_bytes=1 << 30, slots=1, small_n=0).run([r])
    torch.cuda.synchronize()
    for a, b in zip(mix, alone):
        assert np.array_equal(to_host(a.result), to_host(b.result)), (a.rid, a.kind, a.n)
