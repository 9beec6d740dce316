"""Serving loop logic on the CPU (fake executor, virtual clock): FIFO
admission by memory footprint, back-pressure, slot limits, grouping of small
products, rejection of oversize requests, and an injected executor failure
that fails only its own batch."""
import numpy as np

from paper_1510_08642_amd import inputs
from paper_1510_08642_amd.serve import Request, Server, make_requests
from tests.fake_executor import FakeExecutor, VirtualClock


def reqs_from(spec):
    return [Request(rid=i, kind=k, n=n, nrhs=r, t_arrive=t) for i, (k, n, r, t) in enumerate(spec)]


def test_all_complete_and_latency_order():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    trace = inputs.serving_trace(200, rate=2000.0, seed=3, gemm_n=(8, 64), lu_n=(8, 64),
                                 nrhs=(1, 4))
    reqs = make_requests(trace)
    st = Server(ex, budget_bytes=10 ** 9, slots=4, small_n=32).run(reqs, clock=clock)
    assert st.completed == 200 and st.failed == 0
    assert all(r.t_done >= r.t_admit >= r.t_arrive for r in reqs)
    assert st.p99_ms >= st.p50_ms > 0
    assert ex.max_concurrent <= 4


def test_budget_is_never_exceeded_and_backpressure_waits():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    # each n=100 product needs 16*100*100 + 16*100 bytes; the budget fits two
    fp = 16 * 100 * 100 + 16 * 100
    reqs = reqs_from([("gemm", 100, 0, 0.0)] * 6)
    srv = Server(ex, budget_bytes=2 * fp + 10, slots=8, small_n=0)
    st = srv.run(reqs, clock=clock)
    assert st.completed == 6
    assert st.max_inflight_bytes <= 2 * fp + 10
    assert ex.max_concurrent == 2           # memory, not slots, limited concurrency
    # FIFO: admission times are non-decreasing in request order
    ta = [r.t_admit for r in reqs]
    assert ta == sorted(ta)


def test_small_products_are_grouped():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    reqs = reqs_from([("gemm", 16, 0, 0.0)] * 10 + [("lu", 16, 2, 0.0)] + [("gemm", 16, 0, 0.0)] * 5)
    st = Server(ex, budget_bytes=10 ** 9, slots=2, small_n=32, max_batch=8).run(reqs, clock=clock)
    assert st.completed == 16
    sizes = [len(b) for b, _, _ in ex.launched]
    assert max(sizes) == 8
    # the LU request is never merged with products
    for b, _, _ in ex.launched:
        kinds = {reqs[i].kind for i in b}
        assert len(kinds) == 1
        assert kinds == {"gemm"} or len(b) == 1


def test_oversize_rejected_and_injected_failure_isolated():
    clock = VirtualClock()
    ex = FakeExecutor(clock, fail_rids={2})
    reqs = reqs_from([("gemm", 20, 0, 0.0), ("gemm", 4000, 0, 0.0), ("lu", 20, 1, 0.0),
                      ("gemm", 20, 0, 0.0)])
    st = Server(ex, budget_bytes=10 ** 6, slots=1, small_n=0).run(reqs, clock=clock)
    assert reqs[1].error and "budget" in reqs[1].error
    assert reqs[2].error and "injected" in reqs[2].error
    assert reqs[0].error is None and reqs[3].error is None
    assert st.completed == 2 and st.failed == 2


def test_results_flow_through_with_oracle_payloads():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    g = inputs.rng(5)
    reqs = reqs_from([("gemm", 12, 0, 0.0), ("lu", 10, 2, 0.0), ("gemm", 9, 0, 0.001)])
    reqs[0].payload = (inputs.dd_uniform(12, 12, g), inputs.dd_uniform(12, 12, g))
    reqs[1].payload = (inputs.dd_lu_matrix(10, g), inputs.dd_uniform(10, 2, g))
    reqs[2].payload = (inputs.dd_uniform(9, 9, g), inputs.dd_uniform(9, 9, g))
    Server(ex, budget_bytes=10 ** 7, slots=2, small_n=16).run(reqs, clock=clock)
    A, B = reqs[0].payload
    assert np.allclose(reqs[0].result[0], A[0] @ B[0])
    A, B = reqs[1].payload
    assert np.allclose(A[0] @ reqs[1].result[0], B[0])


def test_online_server_futures_from_threads():
    """The live front end: submissions from several threads, answers through
    futures, equal to the oracle's direct results; an oversize request and an
    injected failure fail only their own futures."""
    import threading

    import oracle
    from paper_1510_08642_amd.serve import OnlineServer

    clock = VirtualClock()
    ex = FakeExecutor(clock, fail_rids={3})
    srv = OnlineServer(ex, budget_bytes=10 ** 6, slots=2, small_n=0, clock=clock,
                       idle_sleep_s=0.0)
    g = inputs.rng(9)
    jobs = [("gemm", inputs.dd_uniform(12, 12, g), inputs.dd_uniform(12, 12, g)),
            ("lu", inputs.dd_lu_matrix(10, g), inputs.dd_uniform(10, 3, g)),
            ("gemm", inputs.dd_uniform(7, 7, g), inputs.dd_uniform(7, 7, g)),
            ("gemm", inputs.dd_uniform(5, 5, g), inputs.dd_uniform(5, 5, g)),
            ("gemm", inputs.dd_uniform(9, 9, g), inputs.dd_uniform(9, 9, g))]
    futs = [None] * len(jobs)

    def submit(k):
        kind, A, B = jobs[k]
        futs[k] = srv.submit_gemm(A, B) if kind == "gemm" else srv.submit_lu_solve(A, B)
    # request ids follow submission order; submit 0..2 from threads, then 3, 4
    for k in range(3):
        t = threading.Thread(target=submit, args=(k,))
        t.start()
        t.join()
    submit(3)
    submit(4)
    big = srv.submit_gemm(np.zeros((2, 400, 400)), np.zeros((2, 400, 400)))
    for k, (kind, A, B) in enumerate(jobs):
        if k == 3:
            try:
                futs[k].result(timeout=30)
                raise AssertionError("the injected failure must surface")
            except RuntimeError as e:
                assert "injected" in str(e)
            continue
        got = futs[k].result(timeout=30)
        if kind == "gemm":
            assert np.array_equal(got, oracle.gemm(A, B, "block"))
        else:
            LU, ipiv, _ = oracle.getrf(A, panel=8)
            assert np.array_equal(got, oracle.getrs(LU, ipiv, B))
    try:
        big.result(timeout=30)
        raise AssertionError("oversize request must fail")
    except RuntimeError as e:
        assert "budget" in str(e)
    srv.close(timeout=30)
    st = srv.stats()
    assert st.completed == 4 and st.failed == 2


def test_blocked_head_is_bypassed_by_requests_that_fit():
    """A head that does not fit the free memory lets a later small request go
    first (the loop stays busy); with max_bypass = 0 admission is strictly
    oldest first."""
    fp_big = 16 * 300 * 300 + 16 * 300
    for max_bypass, expect_small_first in ((8, True), (0, False)):
        clock = VirtualClock()
        ex = FakeExecutor(clock)
        reqs = reqs_from([("gemm", 300, 0, 0.0), ("gemm", 300, 0, 0.0), ("gemm", 10, 0, 0.0)])
        Server(ex, budget_bytes=fp_big + 5000, slots=4, small_n=0,
               max_bypass=max_bypass).run(reqs, clock=clock)
        assert all(r.error is None for r in reqs)
        small_first = reqs[2].t_admit < reqs[1].t_admit
        assert small_first == expect_small_first, max_bypass
        if expect_small_first:
            assert reqs[1].bypassed >= 1


def test_bypass_is_bounded():
    """A head passed max_bypass times waits until it fits: no starvation by a
    stream of small requests."""
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    fp_big = 16 * 300 * 300 + 16 * 300
    spec = [("gemm", 300, 0, 0.0), ("gemm", 300, 0, 0.0)] + [("gemm", 10, 0, 0.0)] * 40
    reqs = reqs_from(spec)
    Server(ex, budget_bytes=fp_big + 5000, slots=4, small_n=0, max_bypass=5).run(reqs,
                                                                            clock=clock)
    head = reqs[1]
    assert head.bypassed == 5
    passed = [r for r in reqs[2:] if r.t_admit < head.t_admit]
    assert len(passed) == 5


def test_reserved_slot_keeps_small_requests_flowing():
    """With one of two slots reserved for small requests, two large
    factorizations run one at a time and the small products use the other
    slot meanwhile."""
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    reqs = reqs_from([("lu", 600, 4, 0.0), ("lu", 600, 4, 0.0)] +
                     [("gemm", 20, 0, 0.0)] * 6)
    Server(ex, budget_bytes=10 ** 9, slots=2, small_n=0, reserve_small=1,
           small_flops=2.0 * 64 ** 3).run(reqs, clock=clock)
    big0, big1 = reqs[0], reqs[1]
    assert big1.t_admit >= big0.t_done - 1e-9        # never both large ones at once
    smalls = reqs[2:]
    assert all(r.t_done <= big0.t_done for r in smalls)   # they ran beside the first
