#!/usr/bin/env python3
"""Benchmark: DD GEMM effective GFLOPS (2mnl/t) at m = n = l = 1024 on one GPU.

One step is one double-double product C := A B at n = 1024 (inputs: DD
uniform, seed 0, already resident in HBM) through the library's C ABI with
the flagship configuration.  After W warm-up steps, K steps are timed with
HIP events on the stream the kernels run on, bracketed by device
synchronisation.  Rank 0 prints one JSON line.

Also reported in the same line:
  * roofline: the dominant kernel's achieved FP64-operation (or INT8-MFMA)
    rate against the chip's peak, from its own launch durations;
  * variants: every algorithm / base at n = 1024 (and QD), effective GFLOPS;
  * cpu_baseline: the CPU oracle (plain C, OpenMP) on a bounded sample of the
    same workload, on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# MI355X: 256 CUs x 2.4 GHz x 64 FP64 lanes = 39.3e12 FP64 VALU operations/s
# (the 78.6 TFLOP/s datasheet figure counts an FMA as two).
FP64_OPS_PEAK_T = 256 * 2.4e9 * 64 / 1e12
INT8_PEAK_T = 5000.0        # dense INT8 MFMA, TOP/s
# FP64 VALU operations per DD multiply-add in the Block FMA kernel
# (1 mul + 3 fma + 8 add), plus one TwoSum (6 ops) per 16 multiply-adds.
DD_OPS_PER_MAC = 12 + 6 / 16
# per QD multiply-add in the QD Block kernel (see qd_mac), plus renormalise
QD_OPS_PER_MAC = 113 + 30 / 16


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE, WRITE_SIZE scaled by a plain copy's readings), or
    None when the kernel's source has changed since they were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "profiles", "traffic.json")) as f:
            rec = json.load(f)[kernel]
        with open(os.path.join(root, rec["source"]), "rb") as f:
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
    return ev0.elapsed_time(ev1) / steps          # ms per step


def cpu_baseline(n: int, budget_s: float = 20.0):
    """The oracle's Block DD product on a row sample of the n x n workload."""
    import oracle
    from paper_1510_08642_amd import inputs
    g = inputs.rng(0)
    A = inputs.dd_uniform(n, n, g)
    B = inputs.dd_uniform(n, n, g)
    cores = len(os.sched_getaffinity(0))
    rows = 64
    t0 = time.perf_counter()
    oracle.gemm(A[:, :rows], B, "block")
    t = time.perf_counter() - t0
    # grow the sample towards the budget (bounded by the full matrix)
    rows2 = int(min(n, max(rows, rows * budget_s / max(t, 1e-3) / 2)))
    rows2 = max(64, rows2 // 64 * 64)
    t0 = time.perf_counter()
    oracle.gemm(A[:, :rows2], B, "block")
    t = time.perf_counter() - t0
    gf = 2.0 * rows2 * n * n / t / 1e9
    return {"value": round(gf, 4), "unit": "GFLOPS", "cores": cores, "kind": "oracle",
            "sample": f"oracle Block DD product of the first {rows2} rows of A (n={n}) by B, "
                      f"{t:.2f} s on {cores} threads (OpenMP over row blocks)"}


def sampled_error(A, B, C, n, count=64):
    """Row-normwise error of C on sampled entries against the oracle's exact
    product."""
    import oracle
    g = np.random.default_rng(0)
    ii = g.integers(0, n, count)
    jj = g.integers(0, n, count)
    e = np.abs(oracle.exact_error(A, B, C, ii, jj))
    den = (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)[ii]
    return float(np.max(e / den))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--algo", default="block")
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--base", default="fma")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB, 5 times "
                         "(reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
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
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1510_08642_amd import ddqd, inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    n = args.n
    g = inputs.rng(0)
    A = torch.from_numpy(inputs.dd_uniform(n, n, g)).to(dev)
    B = torch.from_numpy(inputs.dd_uniform(n, n, g)).to(dev)
    C = torch.empty((2, n, n), dtype=torch.float64, device=dev)

    def make(algo, levels, base, P=2, X=A, Y=B, Z=C):
        ws = torch.empty(max(1, ddqd.gemm_workspace(P, n, n, n, algo, levels, base)),
                         dtype=torch.uint8, device=dev)
        f = ddqd.dd_gemm if P == 2 else ddqd.qd_gemm
        if P == 2:
            return lambda: f(X, Y, Z, algo=algo, levels=levels, base=base, ws=ws)
        return lambda: f(X, Y, Z, algo=algo, levels=levels, ws=ws)

    log(f"bench: n={n} algo={args.algo} levels={args.levels} base={args.base}")
    step = make(args.algo, args.levels, args.base)
    ms = time_steps(step, args.steps, args.warmup, stream)
    flops = 2.0 * n * n * n
    value = flops / (ms * 1e-3) / 1e9
    log(f"bench: {ms:.3f} ms/step, {value:.1f} GFLOPS effective")

    # roofline of the dominant kernel (the leaf product)
    if args.base == "fma" and (args.algo == "block" or
                               (args.algo in ("strassen", "winograd") and args.levels == 0)):
        macs = float(n) ** 3
        achieved = macs * DD_OPS_PER_MAC / (ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "dd_gemm_block_kernel", "achieved": round(achieved, 3),
                "peak": round(FP64_OPS_PEAK_T, 2), "unit": "TFLOP/s",
                "frac": round(achieved / FP64_OPS_PEAK_T, 4),
                "traffic": measured_traffic("dd_gemm_block_kernel"),
                "note": "FP64 VALU operations (add, mul or fma count 1 each; "
                        f"{DD_OPS_PER_MAC} per DD multiply-add) over the kernel's "
                        "average launch time; peak = 256 CU x 2.4 GHz x 64 lanes"}
    else:
        roof = None

    variants = {}
    if not args.no_variants:
        for (algo, lv, base) in [("block", 0, "fma"), ("strassen", 1, "fma"),
                                 ("strassen", 2, "fma"), ("strassen", 3, "fma"),
                                 ("winograd", 1, "fma"), ("winograd", 2, "fma"),
                                 ("winograd", 3, "fma"), ("block", 0, "ozaki"),
                                 ("winograd", 1, "ozaki"), ("winograd", 2, "ozaki"),
                                 ("strassen", 1, "ozaki")]:
            try:
                t = time_steps(make(algo, lv, base), max(3, args.steps // 4), 1, stream)
                variants[f"dd_{algo}{lv}_{base}"] = round(flops / (t * 1e-3) / 1e9, 1)
                log(f"variant dd {algo} L{lv} {base}: {t:.3f} ms")
            except Exception as ex:
                variants[f"dd_{algo}{lv}_{base}"] = f"error: {ex}"
        gq = inputs.rng(0)
        Aq = torch.from_numpy(inputs.qd_uniform(n, n, gq)).to(dev)
        Bq = torch.from_numpy(inputs.qd_uniform(n, n, gq)).to(dev)
        Cq = torch.empty((4, n, n), dtype=torch.float64, device=dev)
        for (algo, lv) in [("block", 0), ("winograd", 1), ("winograd", 3)]:
            t = time_steps(make(algo, lv, "fma", 4, Aq, Bq, Cq), 2, 1, stream)
            variants[f"qd_{algo}{lv}_fma"] = round(flops / (t * 1e-3) / 1e9, 1)
            log(f"variant qd {algo} L{lv}: {t:.3f} ms")

    # CPU-baseline leg: the oracle timed on this host, and the oracle's exact
    # product used to state the timed result's error on sampled entries
    cpu, err = None, None
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        cpu = cpu_baseline(n)
        log(f"bench: cpu baseline {cpu}")
        step()
        torch.cuda.synchronize()
        err = sampled_error(A.cpu().numpy(), B.cpu().numpy(), C.cpu().numpy(), n)
        log(f"bench: sampled row-normwise error {err:.3e} (tolerance {2.0**-100*n:.3e})")

    out = {
        "metric": "DD GEMM effective GFLOPS (2mnl/t) at n=1024",
        "value": round(value, 2), "unit": "GFLOPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dd_gemm m=n=l={n}, DD uniform seed 0",
                   "algo": args.algo, "levels": args.levels, "base": args.base,
                   "parallelism": "single GPU"},
        "error_rownorm": err,
        "roofline": roof,
        "variants_gflops": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
