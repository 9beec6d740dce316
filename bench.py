#!/usr/bin/env python3
"""Benchmark: DD GEMM effective GFLOPS (2mnl/t) at m = n = l = 1024 on one GPU,
with DD LU and the serving loop's p50/p99 latency beside it.

Step: one double-double product C := A B at n = 1024 (DD uniform inputs,
seed 0, resident in HBM before timing) through the C ABI with the flagship
configuration (Block algorithm on the CRT INT8-MFMA base: 30 moduli, one
exact INT8 product each, the integer product rebuilt by the Chinese
remainder theorem; its accuracy matches the FMA base).  W warm-up steps, then K steps timed with HIP
events on the stream the library launches on, bracketed by device
synchronisation; rank 0 prints one JSON line.

Also in the line:
  roofline      the dominant kernel's achieved rate against MI355X's peak,
                from its own launch durations (library event hooks, a second
                pass of the same K steps so the main timing carries no events)
  roofline_ozaki the Ozaki split's product kernel (the other INT8 base)
  variants      every algorithm / base for DD at n = 1024, and QD
  lu            dd_getrf / dd_getrs at n = 2048 and 4096 (N(0,1) + n I)
  serving       2000 Poisson requests (60 % DD products, n log-uniform in
                [64, 1024]; 40 % LU factor + solve, n in [128, 2048], 1-16
                right-hand sides) at 50 % and 90 % of the measured capacity,
                FMA vs Ozaki base: p50 / p99 latency and throughput
  cpu_baseline  the CPU oracle on a bounded sample of the step's workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# MI355X peaks.  FP64 VALU: 256 CUs x 2.4 GHz x 64 lanes = 39.3e12 operations/s
# (add, mul or fma counting one; the 78.6 TFLOP/s datasheet figure counts an
# FMA as two).  INT8 matrix cores: 5.0 POP/s dense (datasheet).
FP64_OPS_PEAK_T = 256 * 2.4e9 * 64 / 1e12
INT8_PEAK_T = 5000.0
# FP64 operations per DD multiply-add of the Block FMA kernel (1 mul + 3 fma +
# 8 add, and a 6-operation TwoSum every 16) -- confirmed by SQ_INSTS_VALU_*_F64
DD_OPS_PER_MAC = 12 + 6 / 16
# FP64 operations per QD multiply-add of the QD Block FMA kernel (six
# TwoProducts, four order-3 products, 14 TwoSums and 13 adds = 113, and a
# 30-operation renormalisation every 16) -- SQ_INSTS_VALU_*_F64 counts 114.91
QD_OPS_PER_MAC = 113 + 30 / 16


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, or None if the
    kernel's source changed since (FETCH_SIZE and WRITE_SIZE, scaled by what
    the same counters read for a plain copy of known size)."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f)[kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
                return None
        return int(1024 * (rec["fetch_kib"] * rec["fetch_scale"] +
                           rec["write_kib"] * rec["write_scale"]))
    except (OSError, KeyError, ValueError):
        return None


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def kernel_avg_ms(dd, fn, steps, name):
    """Average duration of the library's kernels named `name` over `steps`
    calls of fn, from the library's own event hooks (recorded on the stream
    each kernel is launched on)."""
    import torch
    torch.cuda.synchronize()
    dd.profile_reset()
    dd.profile_enable(True)
    for _ in range(steps):
        fn()
    dd.profile_enable(False)
    ms, cnt = dd.profile_query(name)
    dd.profile_reset()
    return ms / max(cnt, 1), cnt


def roofline(dd, args, n, step, steps):
    leaves = 7 ** args.levels if args.algo in ("strassen", "winograd") else 1
    lf = n // (2 ** args.levels) if leaves > 1 else n
    if args.base == "crt":
        name = "crt_gemm_kernel"
        qd = args.precision == "qd"
        N = len(dd.crt_moduli(lf, precision=4 if qd else 2))
        avg, cnt = kernel_avg_ms(dd, step, steps, name)
        per = max(1, cnt // steps)
        # QD: H_a H_b over K and the cross product over 2 K per modulus
        ops = 2.0 * lf ** 3 * N * (3 if qd else 1) * leaves / per
        ach = ops / (avg * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": round(ach, 1), "peak": INT8_PEAK_T,
                "unit": "TFLOP/s", "frac": round(ach / INT8_PEAK_T, 4),
                "traffic": measured_traffic(name), "avg_launch_ms": round(avg, 5),
                "launches_per_step": per,
                "note": f"INT8 MFMA operations (2 per multiply-add) of the N = {N} residue "
                        "products per launch (one per modulus); peak = MI355X dense INT8 "
                        "5.0 POP/s"}
    if args.base == "ozaki":
        name, S = "oz_gemm_kernel", 16
        avg, cnt = kernel_avg_ms(dd, step, steps, name)
        per = max(1, cnt // steps)
        ops = 2.0 * lf ** 3 * S * (S + 1) / 2 * leaves / per
        ach = ops / (avg * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": round(ach, 1), "peak": INT8_PEAK_T,
                "unit": "TFLOP/s", "frac": round(ach / INT8_PEAK_T, 4),
                "traffic": measured_traffic(name), "avg_launch_ms": round(avg, 5),
                "launches_per_step": per,
                "note": "INT8 MFMA operations (2 per multiply-add) of the S(S+1)/2 = 136 slice "
                        "products per launch; peak = MI355X dense INT8 5.0 POP/s (a register-only "
                        "microbenchmark of the same MFMA pattern on random data reaches 3.58)"}
    name = "dd_gemm_block_kernel" if args.algo != "simple" else "dd_gemm_simple_kernel"
    avg, cnt = kernel_avg_ms(dd, step, steps, name)
    per = max(1, cnt // steps)
    macs = float(lf) ** 3 * leaves / per
    ach = macs * DD_OPS_PER_MAC / (avg * 1e-3) / 1e12
    return {"bound": "alu", "kernel": name, "achieved": round(ach, 3),
            "peak": round(FP64_OPS_PEAK_T, 2), "unit": "TFLOP/s",
            "frac": round(ach / FP64_OPS_PEAK_T, 4), "traffic": measured_traffic(name),
            "avg_launch_ms": round(avg, 5), "launches_per_step": per,
            "note": f"FP64 VALU operations ({DD_OPS_PER_MAC} per DD multiply-add, each add/mul/"
                    "fma counting one); peak = 256 CU x 2.4 GHz x 64 lanes"}


def roofline_qd_ozaki(dd, step, n, steps, S=31):
    """The QD Ozaki product kernel at n (Block, one leaf): INT8 MFMA operations
    of its S(S+1)/2 slice products against the dense INT8 peak."""
    name = "ozq_gemm_kernel"
    avg, cnt = kernel_avg_ms(dd, step, steps, name)
    per = max(1, cnt // steps)
    ops = 2.0 * n ** 3 * S * (S + 1) / 2 / per
    ach = ops / (avg * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": name, "achieved": round(ach, 1), "peak": INT8_PEAK_T,
            "unit": "TFLOP/s", "frac": round(ach / INT8_PEAK_T, 4),
            "traffic": measured_traffic(name), "avg_launch_ms": round(avg, 5),
            "launches_per_step": per,
            "note": f"qd_gemm base=ozaki, S = {S}: {S * (S + 1) // 2} INT8 slice products "
                    "per launch"}


def roofline_qd_fma(dd, step, n, steps):
    """The QD Block FMA product kernel at n: FP64 VALU operations of its
    multiply-adds against the FP64 issue peak."""
    name = "qd_gemm_block_kernel"
    avg, cnt = kernel_avg_ms(dd, step, steps, name)
    per = max(1, cnt // steps)
    ach = float(n) ** 3 / per * QD_OPS_PER_MAC / (avg * 1e-3) / 1e12
    return {"bound": "alu", "kernel": name, "achieved": round(ach, 3),
            "peak": round(FP64_OPS_PEAK_T, 2), "unit": "TFLOP/s",
            "frac": round(ach / FP64_OPS_PEAK_T, 4), "traffic": measured_traffic(name),
            "avg_launch_ms": round(avg, 5), "launches_per_step": per,
            "note": f"qd_gemm base=fma: FP64 VALU operations ({QD_OPS_PER_MAC} per QD "
                    "multiply-add, each add/mul/fma counting one); peak = 256 CU x 2.4 GHz x "
                    "64 lanes"}


def cpu_baseline(n: int, budget_s: float = 8.0, P: int = 2):
    """The oracle (as it stands) on this host, on bounded samples of the
    workloads: the Block product (DD, or QD for P = 4) of the n x n step
    repeated on all threads for about budget_s seconds (the reported value);
    one thread on a 64-row sample (median of 3); the QD Block product on row
    samples (all threads, one thread); the blocked LU with partial pivoting
    (DD n = 512, QD n = 128; all threads and one thread)."""
    import oracle
    from paper_1510_08642_amd import inputs
    g = inputs.rng(0)
    gen = inputs.dd_uniform if P == 2 else inputs.qd_uniform
    A = gen(n, n, g)
    B = gen(n, n, g)
    threads = oracle.num_threads()

    def timed(fn, reps=1):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def one_thread(fn, reps=1):
        oracle.set_threads(1)
        try:
            return timed(fn, reps)
        finally:
            oracle.set_threads(threads)

    reps, t = 0, 0.0
    while t < budget_s or reps == 0:
        t += timed(lambda: oracle.gemm(A, B, "block"))
        reps += 1
    gf = 2.0 * n ** 3 * reps / t / 1e9
    rows = 64
    t1 = one_thread(lambda: oracle.gemm(A[:, :rows], B, "block"), reps=3)
    gf1 = 2.0 * rows * n * n / t1 / 1e9
    # QD: the oracle's exact-expansion arithmetic is slow, so row samples
    # (block size 4 so that every thread gets rows)
    Aq = inputs.qd_uniform(32, n, g)
    Bq = inputs.qd_uniform(n, n, g)
    tq = timed(lambda: oracle.gemm(Aq, Bq, "block", bs=4))
    tq1 = one_thread(lambda: oracle.gemm(Aq[:, :4], Bq, "block", bs=4))
    qd = {"gflops_all_threads": round(2.0 * 32 * n * n / tq / 1e9, 5),
          "gflops_one_thread": round(2.0 * 4 * n * n / tq1 / 1e9, 5),
          "sample": f"QD Block, 32 rows x {n} x {n} on {threads} threads ({tq:.1f} s), "
                    f"4 rows on one thread ({tq1:.1f} s)"}
    lu = {}
    for Pl, nl in ((2, 512), (4, 128)):
        Al = (inputs.dd_lu_matrix if Pl == 2 else inputs.qd_lu_matrix)(nl, g)
        f = lambda: oracle.getrf(Al, panel=64, pivot=True, algo="block", levels=0)
        ta, t1l = timed(f), one_thread(f)
        lu[f"{'dd' if Pl == 2 else 'qd'}_getrf_n{nl}"] = {
            "ms_all_threads": round(ta * 1e3, 1), "ms_one_thread": round(t1l * 1e3, 1),
            "gflops_all_threads": round(2.0 / 3.0 * nl ** 3 / ta / 1e9, 5)}
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(gf, 4), "unit": "GFLOPS", "cores": threads, "kind": "oracle",
            "sample": f"oracle Block {'DD' if P == 2 else 'QD'} product of the whole n={n} "
                      f"workload, {reps} times in {t:.1f} s on {threads} OpenMP threads "
                      f"({model}); one thread on the first {rows} rows: {gf1:.3f} GFLOPS "
                      "(median of 3)",
            "one_thread_gflops": round(gf1, 4), "cpu_model": model, "qd": qd, "lu": lu}


def sampled_error(A, B, C, n, count=64):
    """Row-normwise error of C on sampled entries against the oracle's exact
    product (part of the CPU-baseline leg)."""
    import oracle
    g = np.random.default_rng(0)
    ii = g.integers(0, n, count)
    jj = g.integers(0, n, count)
    e = np.abs(oracle.exact_error(A, B, C, ii, jj))
    den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)[ii]
    return float(np.max(e / den))


def qd_residual(dd, torch, A, x, b):
    """||b - A x||_inf / (||A||_inf ||x||_inf) with the residual evaluated by
    the library's QD product (A, x, b widened to four planes exactly): for a
    DD solve the evaluation's own rounding (about n 2^-212) is far below the
    residual; for a QD solve it is of the residual's order, so the figure is
    an estimate within a small factor."""
    P, n = A.shape[0], A.shape[1]

    def q(X):
        if P == 4:
            return X.contiguous()
        Z = torch.zeros((4,) + tuple(X.shape[1:]), dtype=torch.float64, device=X.device)
        Z[:P] = X
        return Z
    Aq = q(A)
    r = q(b)
    dd.qd_gemm(Aq, q(x), r, alpha=-1, beta=1)
    rh = r[0].abs().max().item()
    normA = A[0].abs().sum(dim=1).max().item()
    normx = x[0].abs().max().item()
    del Aq, r
    return rh / (normA * normx)


def bench_lu(dd, inputs, torch, dev, sizes, configs, stream, P=2):
    out = {}
    getrf = dd.dd_getrf if P == 2 else dd.qd_getrf
    getrs = dd.dd_getrs if P == 2 else dd.qd_getrs
    for n in sizes:
        g = inputs.rng(0)
        A0 = torch.from_numpy((inputs.dd_lu_matrix if P == 2 else inputs.qd_lu_matrix)(n, g)).to(dev)
        b0 = torch.from_numpy((inputs.dd_uniform if P == 2 else inputs.qd_uniform)(n, 16, g)).to(dev)
        for (panel, algo, lv, base) in configs:
            key = ("" if P == 2 else "qd_") + f"n{n}_p{panel}_{algo}{lv}_{base}"
            ws = torch.empty(max(1, dd.getrf_workspace(n, panel, algo, lv, base, P)),
                             dtype=torch.uint8, device=dev)
            A = A0.clone()
            holder = {}

            def f():
                A.copy_(A0)
                holder["f"] = getrf(A, panel=panel, algo=algo, levels=lv, base=base, ws=ws)
            t_copy = time_steps(lambda: A.copy_(A0), 3, 1, stream)
            t_f = time_steps(f, 2, 1, stream)         # A holds the factors after this
            ipiv, perm, _ = holder["f"]
            res = {}
            for nrhs in (1, 16):
                Xs = b0[:, :, :nrhs].contiguous()

                def s():
                    Xs.copy_(b0[:, :, :nrhs])
                    getrs(A, ipiv, Xs, perm=perm)
                res[nrhs] = time_steps(s, 3, 1, stream)
            t_getrf = t_f - t_copy
            # Eq. 2's solve for one right-hand side, and its residual
            x1 = b0[:, :, :1].contiguous()
            getrs(A, ipiv, x1, perm=perm)
            resid = qd_residual(dd, torch, A0, x1, b0[:, :, :1].contiguous())
            out[key] = {"getrf_ms": round(t_getrf, 3),
                        "getrf_gflops": round(2.0 / 3.0 * n ** 3 / (t_getrf * 1e-3) / 1e9, 1),
                        "getrs_ms_nrhs1": round(res[1], 3), "getrs_ms_nrhs16": round(res[16], 3),
                        "residual_nrhs1": float(f"{resid:.3e}"),
                        "residual_bound": float(f"{n * (2.0 ** -100 if P == 2 else 2.0 ** -200):.3e}")}
            log(f"lu {key}: {out[key]}")
    return out


def bench_graphs(dd, inputs, torch, dev):
    """Eager calls against a replay of the same calls recorded as a graph."""
    out = {}
    side = torch.cuda.Stream(dev)

    def timed(fn, reps):
        with torch.cuda.stream(side):
            return time_steps(fn, reps, 2, side)

    # small product (the 128 x 128 x 128 DD case): launch-bound
    g = inputs.rng(5)
    for m in (128, 512):
        A = torch.from_numpy(inputs.dd_uniform(m, m, g)).to(dev)
        B = torch.from_numpy(inputs.dd_uniform(m, m, g)).to(dev)
        C = torch.empty((2, m, m), dtype=torch.float64, device=dev)
        ws = torch.empty(max(1, dd.gemm_workspace(2, m, m, m, "winograd", 1, "fma")),
                         dtype=torch.uint8, device=dev)

        def f():
            dd.dd_gemm(A, B, C, algo="winograd", levels=1, ws=ws)
        gr = dd.capture(f, side)
        e = timed(f, 50)
        r = timed(lambda: gr.replay(side.cuda_stream), 50)
        out[f"dd_gemm_winograd1_n{m}"] = {"eager_ms": round(e, 4), "graph_ms": round(r, 4)}
        gr.release()
    # LU factor + 1-RHS solve at n = 2048
    n = 2048
    kw = dict(panel=128, algo="winograd", levels=1, base="ozaki")
    A0 = torch.from_numpy(inputs.dd_lu_matrix(n, inputs.rng(0))).to(dev)
    b0 = torch.from_numpy(inputs.dd_uniform(n, 1, inputs.rng(1))).to(dev)
    A, b = A0.clone(), b0.clone()
    ws = torch.empty(max(1, dd.getrf_workspace(n, **kw)), dtype=torch.uint8, device=dev)
    rws = torch.empty(max(1, dd.lib().dd_getrs_workspace(n, 1)), dtype=torch.uint8, device=dev)
    piv = tuple(torch.empty(k, dtype=torch.int32, device=dev) for k in (n, n, 1))

    def lu():
        dd.dd_getrf(A, ws=ws, out=piv, **kw)
        dd.dd_getrs(A, piv[0], b, perm=piv[1], ws=rws)
    gr = dd.capture(lu, side)

    def eager():
        A.copy_(A0)
        b.copy_(b0)
        lu()

    def replay():
        A.copy_(A0)
        b.copy_(b0)
        gr.replay(side.cuda_stream)
    out[f"dd_getrf_getrs_n{n}"] = {"eager_ms": round(timed(eager, 3), 3),
                                    "graph_ms": round(timed(replay, 3), 3)}
    gr.release()
    log(f"graphs: {out}")
    return out


def bench_tuning(dd, inputs, torch, dev, n):
    """Autotuned configuration per product kind at n (dd_gemm_tune / qd_gemm_tune)
    and LU panel width at n and 2n (ddqd_getrf_tune)."""
    out = {}
    g = inputs.rng(7)
    A = torch.from_numpy(inputs.dd_uniform(n, n, g)).to(dev)
    B = torch.from_numpy(inputs.dd_uniform(n, n, g)).to(dev)
    for base in ("fma", "ozaki"):
        r = dd.tune(A, B, base=base, reps=3)
        r["gflops"] = round(2.0 * n ** 3 / (r["ms"] * 1e-3) / 1e9, 1)
        r["ms"] = round(r["ms"], 4)
        out[f"dd_{base}_n{n}"] = r
    Aq = torch.from_numpy(inputs.qd_uniform(n, n, g)).to(dev)
    Bq = torch.from_numpy(inputs.qd_uniform(n, n, g)).to(dev)
    for base in ("fma", "ozaki"):
        r = dd.tune(Aq, Bq, base=base, reps=1 if base == "fma" else 3)
        r["gflops"] = round(2.0 * n ** 3 / (r["ms"] * 1e-3) / 1e9, 1)
        r["ms"] = round(r["ms"], 4)
        out[f"qd_{base}_n{n}"] = r
    # LU panel width per order (Sec. 4's K = 32 alpha sweep), Winograd-1 on Ozaki leaves
    for nl in (n, 2 * n):
        Al = torch.from_numpy(inputs.dd_lu_matrix(nl, inputs.rng(0))).to(dev)
        r = dd.getrf_tune(Al, algo="winograd", levels=1, base="ozaki", reps=2)
        r["gflops"] = round(2.0 / 3.0 * nl ** 3 / (r["ms"] * 1e-3) / 1e9, 1)
        r["ms"] = round(r["ms"], 3)
        out[f"lu_dd_winograd1_ozaki_n{nl}"] = r
        del Al
    log(f"tuning: {out}")
    return out


def bench_equal_accuracy(dd, inputs, torch, dev, n, stream):
    """Ozaki slice counts against the FMA form, in DD and in QD: error on
    sampled entries (exact reference from the oracle) and time, so that the
    two forms can be compared at equal accuracy."""
    g = inputs.rng(11)
    out = {}
    for P, cases in ((2, [("fma", 0), ("ozaki", 12), ("ozaki", 13), ("ozaki", 14),
                          ("ozaki", 15), ("ozaki", 16), ("crt", 0)]),
                     (4, [("fma", 0), ("ozaki", 28), ("ozaki", 29), ("ozaki", 30),
                          ("ozaki", 31)])):
        gen = inputs.dd_uniform if P == 2 else inputs.qd_uniform
        A = torch.from_numpy(gen(n, n, g)).to(dev)
        B = torch.from_numpy(gen(n, n, g)).to(dev)
        C = torch.empty((P, n, n), dtype=torch.float64, device=dev)
        Ah, Bh = A.cpu().numpy(), B.cpu().numpy()
        prod = dd.dd_gemm if P == 2 else dd.qd_gemm
        for base, S in cases:
            ws = torch.empty(max(1, dd.gemm_workspace(P, n, n, n, "block", 0, base, S)),
                             dtype=torch.uint8, device=dev)

            def f():
                prod(A, B, C, algo="block", base=base, slices=S, ws=ws)
            t = time_steps(f, 10 if (P == 2 or base != "fma") else 2, 2, stream)
            f()
            torch.cuda.synchronize()
            err = sampled_error(Ah, Bh, C.cpu().numpy(), n)
            key = ("" if P == 2 else "qd_") + f"{base}{S or ''}"
            out[key] = {"ms": round(t, 4), "gflops": round(2.0 * n ** 3 / (t * 1e-3) / 1e9, 1),
                        "error_rownorm": err}
        del A, B, C
    log(f"equal accuracy: {out}")
    return out


def bench_paper(dd, inputs, torch, dev, stream, full=False):
    """The paper's own experiment shapes on this GPU (a few seconds; full=True
    adds Strassen products and the Winograd / Ozaki LU updates).

    Products (Sec. 3, Tables 1-2): the Sec. 3 matrices A = [sqrt5 (i+j-1)],
    B = [sqrt3 (n-i)] at n = 1023, 1024, 1025 in DD and QD, Block against
    Strassen and Winograd with the paper's n_min = 32 (5 levels at n = 1024);
    error = max relative error against the closed form sqrt15 n (n-1)
    (n + 3i - 2) / 6 on sampled entries (mpmath, 400 bits).
    LU (Sec. 4, Fig. 5 upper DD and lower QD): the random matrix with entries
    in [-1, 1], no pivoting, n = 1024, block size K = alpha n_min for
    alpha = 1, ..., 10, trailing update by Block or Winograd (depth down to
    n_min) on the FMA base, and Block on Ozaki leaves; the row-wise parallel
    LU the paper compares against (panel width 0); x = [0, 1, ..., n-1],
    b = A x formed by the library's product, and the maximum relative error of
    the computed x over x_i != 0."""
    import mpmath
    out = {"products": {}, "lu": {}}
    for P in (2, 4):
        for n in (1023, 1024, 1025):
            A, B = inputs.paper_matrices(n, P)
            Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
            C = torch.empty((P, n, n), dtype=torch.float64, device=dev)
            rs = np.random.default_rng(n)
            rows = np.unique(np.concatenate([[0, n // 2, n - 1], rs.integers(0, n, 29)]))
            exact = inputs.paper_product_closed_form(n, rows)
            configs = [("block", 0, "fma"), ("winograd", 5, "fma"), ("block", 0, "ozaki")]
            if full:
                configs.insert(1, ("strassen", 5, "fma"))
            for algo, lv, base in configs:
                ws = torch.empty(max(1, dd.gemm_workspace(P, n, n, n, algo, lv, base)),
                                 dtype=torch.uint8, device=dev)
                if P == 2:
                    f = lambda: dd.dd_gemm(Ad, Bd, C, algo=algo, levels=lv, base=base, ws=ws)
                else:
                    f = lambda: dd.qd_gemm(Ad, Bd, C, algo=algo, levels=lv, base=base, ws=ws)
                t = time_steps(f, 3 if (P == 2 or base == "ozaki") else 1, 1, stream)
                Ch = C.cpu().numpy()
                err = 0.0
                with mpmath.workprec(400):
                    for r, e in zip(rows, exact):
                        for j in (0, n - 1, int(rs.integers(0, n))):
                            v = mpmath.fsum(mpmath.mpf(float(Ch[c, r, j])) for c in range(P))
                            err = max(err, float(abs(v - e) / e))
                key = f"{'dd' if P == 2 else 'qd'}_n{n}_{algo}{lv}_{base}"
                out["products"][key] = {"ms": round(t, 3),
                                        "gflops": round(2.0 * n ** 3 / (t * 1e-3) / 1e9, 1),
                                        "max_rel_error": err}
                log(f"paper {key}: {out['products'][key]}")
            del Ad, Bd, C
    n = 1024
    for P in (2, 4):
        A0 = torch.from_numpy(inputs.paper_random_matrix(n, inputs.rng(0), P)).to(dev)
        x = np.zeros((P, n, 1))
        x[0, :, 0] = np.arange(n)
        prod = dd.dd_gemm if P == 2 else dd.qd_gemm
        getrf = dd.dd_getrf if P == 2 else dd.qd_getrf
        getrs = dd.dd_getrs if P == 2 else dd.qd_getrs
        b = prod(A0, torch.from_numpy(x).to(dev))
        runs = [(0, "rowwise", "fma", 0)]   # the paper's row-wise parallel comparator
        for alpha in range(1, 11):
            updates = (("block", "fma"), ("winograd", "fma"), ("block", "ozaki")) if full else \
                (("block", "fma"),)
            for algo, base in updates:
                lv = 0 if algo == "block" else alpha.bit_length() - 1
                if algo == "winograd" and lv == 0:
                    continue
                runs.append((32 * alpha, algo, base, lv))
        for K, algo, base, lv in runs:
            palgo = "block" if algo == "rowwise" else algo
            ws = torch.empty(max(1, dd.getrf_workspace(n, K, palgo, lv, base, P)),
                             dtype=torch.uint8, device=dev)
            A = A0.clone()
            hold = {}

            def f():
                A.copy_(A0)
                hold["r"] = getrf(A, panel=K, pivot="none", algo=palgo, levels=lv, base=base,
                                  ws=ws)
            t_copy = time_steps(lambda: A.copy_(A0), 3, 1, stream)
            t = time_steps(f, 2, 1, stream) - t_copy  # A holds the factors after this
            ipiv, perm, info = hold["r"]
            X = b.clone()
            getrs(A, ipiv, X, perm=perm)
            Xh = X.cpu().numpy()[:, :, 0]
            d = np.abs((Xh[0, 1:] - np.arange(1, n)) + sum(Xh[c, 1:] for c in range(1, P)))
            key = (f"{'dd' if P == 2 else 'qd'}_lu_n{n}_rowwise" if K == 0 else
                   f"{'dd' if P == 2 else 'qd'}_lu_n{n}_K{K}_{algo}{lv}_{base}")
            out["lu"][key] = {"getrf_ms": round(t, 3), "info": int(info.cpu()[0]),
                              "max_rel_error_x": float(np.max(d / np.arange(1, n))),
                              "normwise_error_x": float(np.max(d) / (n - 1))}
            log(f"paper {key}: {out['lu'][key]}")
        del A0, b
    return out


def bench_serving(nreq, seed=0):
    from paper_1510_08642_amd import inputs, serve
    pools = serve.DevicePools(nmax_gemm=1024, nmax_lu=2048, nrhs_max=16, seed=seed)
    out = {}
    for base in ("fma", "ozaki"):
        ex = serve.GpuExecutor(slots=4, base=base, gemm_algo="block", gemm_levels=0,
                               lu_panel=128, lu_algo="winograd", lu_levels=1)
        # capacity: every request arrives at t = 0
        trace = inputs.serving_trace(nreq, rate=1e9, seed=seed)
        reqs = serve.make_requests(trace)
        for r in reqs:
            r.payload = pools.payload(r)
        st = serve.Server(ex, budget_bytes=8 << 30, slots=4).run(reqs)
        cap = st.throughput_rps
        res = {"capacity_rps": round(cap, 1), "capacity_gflops": round(st.gflops, 1)}
        del reqs
        for frac in (0.5, 0.9):
            trace = inputs.serving_trace(nreq, rate=frac * cap, seed=seed + 1)
            reqs = serve.make_requests(trace)
            for r in reqs:
                r.payload = pools.payload(r)
            st = serve.Server(ex, budget_bytes=8 << 30, slots=4).run(reqs)
            res[f"load{int(frac * 100)}"] = {
                "rate_rps": round(frac * cap, 1), "p50_ms": round(st.p50_ms, 3),
                "p99_ms": round(st.p99_ms, 3), "throughput_rps": round(st.throughput_rps, 1),
                "gflops": round(st.gflops, 1), "completed": st.completed, "failed": st.failed,
                "batches": st.batches}
            del reqs
        out[base] = res
        log(f"serving {base}: {res}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--algo", default="block")
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--base", default="crt")
    ap.add_argument("--precision", choices=("dd", "qd"), default="dd",
                    help="timed product: dd_gemm (default) or qd_gemm (for profiling the QD "
                         "kernels; the extra legs still run as configured)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-lu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--paper", action="store_true",
                    help="the paper's experiment shapes in full (Sec. 3 tables with Strassen, "
                         "Sec. 4 LU with every update); by default a few-second subset runs")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--lu-only", type=int, default=0, metavar="N",
                    help="only time the DD LU factor-and-solve of order N (panel 128, Winograd 1 "
                         "on Ozaki leaves), for kernel traces of the LU")
    ap.add_argument("--latency-probe", action="store_true",
                    help="print the dependent-chain latencies of the LU column step's "
                         "operations (ddqd_latency_probe) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB, 5 times "
                         "(reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (sharding across GPUs is a design, not implemented); --gpus must be 1"}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {nbytes} bytes")
        return
    sys.path.insert(0, ROOT)
    from paper_1510_08642_amd import ddqd as dd
    from paper_1510_08642_amd import inputs
    if args.latency_probe:
        for threads in (64, 256, 1024):
            dd.latency_probe(threads)                 # warm-up
            print(json.dumps({"threads": threads, "ticks_per_step": dd.latency_probe(threads)}))
        return

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.lu_only:
        out = bench_lu(dd, inputs, torch, dev, [args.lu_only], [(128, "winograd", 1, "ozaki")],
                       stream)
        print(json.dumps({"lu": out}))
        return
    n = args.n
    g = inputs.rng(0)
    PM = 2 if args.precision == "dd" else 4
    gen = inputs.dd_uniform if PM == 2 else inputs.qd_uniform
    A = torch.from_numpy(gen(n, n, g)).to(dev)
    B = torch.from_numpy(gen(n, n, g)).to(dev)
    C = torch.empty((PM, n, n), dtype=torch.float64, device=dev)

    def make(algo, levels, base, P=2, X=A, Y=B, Z=C):
        ws = torch.empty(max(1, dd.gemm_workspace(P, n, n, n, algo, levels, base)),
                         dtype=torch.uint8, device=dev)
        if P == 2:
            return lambda: dd.dd_gemm(X, Y, Z, algo=algo, levels=levels, base=base, ws=ws)
        return lambda: dd.qd_gemm(X, Y, Z, algo=algo, levels=levels, base=base, ws=ws)

    log(f"bench: n={n} algo={args.algo} levels={args.levels} base={args.base}")
    step = make(args.algo, args.levels, args.base, PM)
    ms = time_steps(step, args.steps, args.warmup, stream)
    flops = 2.0 * n * n * n
    value = flops / (ms * 1e-3) / 1e9
    log(f"bench: {ms:.4f} ms/step, {value:.1f} GFLOPS effective")
    if PM == 4:
        if args.algo != "block":
            sys.exit("--precision qd times the QD Block product (either base)")
        roof = (roofline_qd_ozaki(dd, step, n, args.steps) if args.base == "ozaki" else
                roofline(dd, args, n, step, args.steps) if args.base == "crt" else
                roofline_qd_fma(dd, step, n, min(args.steps, 5)))
    else:
        roof = roofline(dd, args, n, step, args.steps)
    log(f"bench: roofline {roof}")
    roof_oz = None
    if PM == 2 and args.base != "ozaki":
        oz_args = argparse.Namespace(**{**vars(args), "base": "ozaki"})
        roof_oz = roofline(dd, oz_args, n, make(args.algo, args.levels, "ozaki"), args.steps)
        log(f"bench: Ozaki roofline {roof_oz}")

    variants = {}
    roof_qd = roof_qd_fma = roof_qd_crt = None
    if not args.no_variants:
        for (algo, lv, base) in [("simple", 0, "fma"), ("block", 0, "fma"),
                                 ("strassen", 1, "fma"), ("strassen", 2, "fma"),
                                 ("strassen", 3, "fma"), ("winograd", 1, "fma"),
                                 ("winograd", 2, "fma"), ("winograd", 3, "fma"),
                                 ("block", 0, "ozaki"), ("strassen", 1, "ozaki"),
                                 ("winograd", 1, "ozaki"), ("winograd", 2, "ozaki"),
                                 ("block", 0, "crt"), ("strassen", 1, "crt"),
                                 ("winograd", 1, "crt"), ("winograd", 2, "crt")]:
            t = time_steps(make(algo, lv, base), 5 if algo != "simple" else 2, 1, stream)
            variants[f"dd_{algo}{lv}_{base}"] = round(flops / (t * 1e-3) / 1e9, 1)
            log(f"variant dd {algo} L{lv} {base}: {t:.3f} ms")
        gq = inputs.rng(0)
        Aq = torch.from_numpy(inputs.qd_uniform(n, n, gq)).to(dev)
        Bq = torch.from_numpy(inputs.qd_uniform(n, n, gq)).to(dev)
        Cq = torch.empty((4, n, n), dtype=torch.float64, device=dev)
        for (algo, lv, base) in [("block", 0, "fma"), ("strassen", 1, "fma"),
                                 ("winograd", 1, "fma"), ("winograd", 2, "fma"),
                                 ("winograd", 3, "fma"), ("block", 0, "ozaki"),
                                 ("winograd", 1, "ozaki"), ("block", 0, "crt"),
                                 ("winograd", 1, "crt")]:
            t = time_steps(make(algo, lv, base, 4, Aq, Bq, Cq), 2 if base == "fma" else 5, 1,
                           stream)
            variants[f"qd_{algo}{lv}_{base}"] = round(flops / (t * 1e-3) / 1e9, 1)
            log(f"variant qd {algo} L{lv} {base}: {t:.3f} ms")
        roof_qd = roofline_qd_ozaki(dd, make("block", 0, "ozaki", 4, Aq, Bq, Cq), n, 5)
        log(f"bench: QD Ozaki roofline {roof_qd}")
        roof_qd_fma = roofline_qd_fma(dd, make("block", 0, "fma", 4, Aq, Bq, Cq), n, 2)
        log(f"bench: QD FMA roofline {roof_qd_fma}")
        qd_args = argparse.Namespace(**{**vars(args), "base": "crt", "precision": "qd",
                                        "algo": "block", "levels": 0})
        roof_qd_crt = roofline(dd, qd_args, n, make("block", 0, "crt", 4, Aq, Bq, Cq), 5)
        log(f"bench: QD CRT roofline {roof_qd_crt}")
        del Aq, Bq, Cq

    tuning = equal = None
    row_scaled = None
    if not args.no_variants:
        tuning = bench_tuning(dd, inputs, torch, dev, n)
        if not args.no_cpu:
            equal = bench_equal_accuracy(dd, inputs, torch, dev, n, stream)
        # the DD product at n = 2048: Block, Strassen and Winograd at 1-3
        # levels, FMA against Ozaki leaves
        n2 = 2 * n
        g2 = inputs.rng(3)
        A2 = torch.from_numpy(inputs.dd_uniform(n2, n2, g2)).to(dev)
        B2 = torch.from_numpy(inputs.dd_uniform(n2, n2, g2)).to(dev)
        C2 = torch.empty((2, n2, n2), dtype=torch.float64, device=dev)
        recursive = [("block", 0)] + [(a, lv) for a in ("strassen", "winograd") for lv in (1, 2, 3)]
        for base in ("fma", "ozaki", "crt"):
            for (algo, lv) in recursive:
                ws2 = torch.empty(max(1, dd.gemm_workspace(2, n2, n2, n2, algo, lv, base)),
                                  dtype=torch.uint8, device=dev)
                t = time_steps(lambda: dd.dd_gemm(A2, B2, C2, algo=algo, levels=lv, base=base,
                                                  ws=ws2), 3, 1, stream)
                variants[f"dd_{algo}{lv}_{base}_n{n2}"] = round(2.0 * n2 ** 3 / (t * 1e-3) / 1e9, 1)
                log(f"variant dd {algo} L{lv} {base} n={n2}: {t:.3f} ms")
                del ws2
        del A2, B2, C2
        # the QD product at n = 512 (FMA: Block, Strassen, Winograd at 1-3
        # levels; Block on Ozaki leaves)
        n5 = n // 2
        g5 = inputs.rng(4)
        A5 = torch.from_numpy(inputs.qd_uniform(n5, n5, g5)).to(dev)
        B5 = torch.from_numpy(inputs.qd_uniform(n5, n5, g5)).to(dev)
        C5 = torch.empty((4, n5, n5), dtype=torch.float64, device=dev)
        for (algo, lv, base) in [(a, l, "fma") for (a, l) in recursive] + [("block", 0, "ozaki")]:
            ws5 = torch.empty(max(1, dd.gemm_workspace(4, n5, n5, n5, algo, lv, base)),
                              dtype=torch.uint8, device=dev)
            t = time_steps(lambda: dd.qd_gemm(A5, B5, C5, algo=algo, levels=lv, base=base,
                                              ws=ws5), 3, 1, stream)
            variants[f"qd_{algo}{lv}_{base}_n{n5}"] = round(2.0 * n5 ** 3 / (t * 1e-3) / 1e9, 1)
            log(f"variant qd {algo} L{lv} {base} n={n5}: {t:.3f} ms")
        del A5, B5, C5
        # the row-scaled variant (row i of A times 2^r_i, r_i in [-30, 30]):
        # time here, error in the CPU leg
        As = torch.from_numpy(inputs.row_scaled(A.cpu().numpy() if PM == 2 else
                                                inputs.dd_uniform(n, n, inputs.rng(0)),
                                                inputs.rng(1))[0]).to(dev)
        Cs = torch.empty((2, n, n), dtype=torch.float64, device=dev)
        Bs = B if PM == 2 else torch.from_numpy(inputs.dd_uniform(n, n, inputs.rng(2))).to(dev)
        row_scaled = {}
        for (algo, lv, base) in [("block", 0, "fma"), ("winograd", 1, "fma"),
                                 ("block", 0, "ozaki"), ("winograd", 1, "ozaki"),
                                 ("block", 0, "crt"), ("winograd", 1, "crt")]:
            wss = torch.empty(max(1, dd.gemm_workspace(2, n, n, n, algo, lv, base)),
                              dtype=torch.uint8, device=dev)
            t = time_steps(lambda: dd.dd_gemm(As, Bs, Cs, algo=algo, levels=lv, base=base,
                                              ws=wss), 5, 1, stream)
            row_scaled[f"{algo}{lv}_{base}"] = {"ms": round(t, 4),
                                                "gflops": round(flops / (t * 1e-3) / 1e9, 1),
                                                "C": Cs.clone() if not args.no_cpu else None}
            log(f"row-scaled 2^+-30 dd {algo} L{lv} {base}: {t:.3f} ms")

    graphs = None if args.no_lu else bench_graphs(dd, inputs, torch, dev)

    lu = None
    if not args.no_lu:
        lu = bench_lu(dd, inputs, torch, dev, [2048, 4096],
                      [(128, "winograd", 1, "fma"), (128, "winograd", 1, "ozaki"),
                       (128, "winograd", 1, "crt"), (256, "block", 0, "ozaki")], stream)
        lu.update(bench_lu(dd, inputs, torch, dev, [1024, 2048],
                           [(64, "block", 0, "fma"), (128, "block", 0, "ozaki"),
                            (128, "block", 0, "crt")], stream, P=4))

    paper = None if args.no_paper else bench_paper(dd, inputs, torch, dev, stream, full=args.paper)

    serving = None
    if not args.no_serving and args.serving_requests > 0:
        serving = bench_serving(args.serving_requests)

    # CPU-baseline leg: the oracle timed on this host, and the oracle's exact
    # product stating the timed result's error on sampled entries
    cpu, err = None, None
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        cpu = cpu_baseline(n, P=PM)
        log(f"bench: cpu baseline {cpu}")
        step()
        torch.cuda.synchronize()
        err = sampled_error(A.cpu().numpy(), B.cpu().numpy(), C.cpu().numpy(), n)
        tol = (2.0 ** -100 if PM == 2 else 2.0 ** -200) * n
        log(f"bench: sampled row-normwise error {err:.3e} (tolerance {tol:.3e})")
        if row_scaled:
            Ash, Bsh = As.cpu().numpy(), Bs.cpu().numpy()
            for k, v in row_scaled.items():
                v["error_rownorm"] = sampled_error(Ash, Bsh, v.pop("C").cpu().numpy(), n)
            log(f"bench: row-scaled variant {row_scaled}")
    elif row_scaled:
        for v in row_scaled.values():
            v.pop("C", None)

    out = {
        "metric": "DD/QD GEMM effective GFLOPS (2mnl/t) at n=1024; DD LU-solve p50/p99 latency",
        "value": round(value, 2), "unit": "GFLOPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ({"ozaki": "i8 mfma (i32 sums) + f64 recombination",
                   "crt": "i8 mfma (i32 sums) + crt rebuild (%d-bit fixed point) + f64"
                          % (160 if PM == 2 else 270)}
                  .get(args.base, "f64")),
        "data": "synthetic",
        "config": {"workload": f"{args.precision}_gemm m=n=l={n}, "
                               f"{args.precision.upper()} uniform inputs seed 0",
                   "algo": args.algo, "levels": args.levels, "base": args.base,
                   "slices": (16 if PM == 2 else 31) if args.base == "ozaki" else None,
                   "moduli": (len(dd.crt_moduli(n, precision=PM)) if args.base == "crt"
                              else None)},
        "error_rownorm": err,
        "roofline": roof,
        "roofline_ozaki": roof_oz,
        "roofline_qd_ozaki": roof_qd,
        "roofline_qd_fma": roof_qd_fma,
        "roofline_qd_crt": roof_qd_crt,
        "variants_gflops": variants,
        "tuned": tuning,
        "ozaki_vs_fma_equal_accuracy": equal,
        "row_scaled_2pm30": row_scaled,
        "graphs": graphs,
        "lu": lu,
        "serving": serving,
        "paper_replication": paper,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
