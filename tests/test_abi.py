"""C-ABI contract of libddqd.so, checked without a GPU.

The library must load here (ROCm is installed), export every function that
include/ddqd.h declares, and reject bad arguments with the documented status
before touching any device.  No call here reaches a kernel launch.
"""
import ctypes
import os
import re

import pytest

from tests.helpers import on_gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1510_08642_amd", "libddqd.so")
HEADER = os.path.join(ROOT, "include", "ddqd.h")

E = dict(OK=0, ARG=1, ALIAS=2, WORKSPACE=3, UNSUPPORTED=4, NODEVICE=5, HIP=6)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1510_08642_amd import build
        build.build()
    from paper_1510_08642_amd import ddqd
    return ddqd.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for want in ["dd_gemm", "dd_gemm_workspace", "qd_gemm", "qd_gemm_workspace",
                 "ddqd_status_string", "ddqd_last_error"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in E.values():
        s = lib.ddqd_status_string(code).decode()
        assert s.startswith("DDQD_")
    assert lib.ddqd_status_string(99).decode() == "unknown status"


def _call(lib, fn="dd_gemm", m=4, n=4, l=4, alpha=1, A=0x10000, lda=4, psa=16, B=0x20000,
          ldb=4, psb=16, beta=0, C=0x30000, ldc=4, psc=16, algo=1, levels=0, base=0, slices=0,
          ws=None, ws_bytes=0):
    return getattr(lib, fn)(m, n, l, alpha, A, lda, psa, B, ldb, psb, beta, C, ldc, psc, algo,
                            levels, base, slices, ws, ws_bytes, None)


@pytest.mark.parametrize("fn", ["dd_gemm", "qd_gemm"])
def test_argument_errors(lib, fn):
    P = 2 if fn == "dd_gemm" else 4
    kw = dict(fn=fn)
    assert _call(lib, m=-1, **kw) == E["ARG"]
    assert _call(lib, alpha=2, **kw) == E["ARG"]
    assert _call(lib, beta=3, **kw) == E["ARG"]
    assert _call(lib, algo=7, **kw) == E["ARG"]
    assert _call(lib, levels=9, **kw) == E["ARG"]
    assert _call(lib, base=5, **kw) == E["ARG"]
    assert _call(lib, lda=3, **kw) == E["ARG"]
    assert _call(lib, ldc=2, **kw) == E["ARG"]
    assert _call(lib, psa=10, **kw) == E["ARG"]
    assert _call(lib, A=0, **kw) == E["ARG"]
    assert _call(lib, C=0x30004, **kw) == E["ARG"]       # misaligned
    assert b"C is not 8-byte aligned" in lib.ddqd_last_error()
    # C overlapping A
    assert _call(lib, C=0x10000 + 8, **kw) == E["ALIAS"]
    # workspace for a Strassen level is required
    assert _call(lib, algo=2, levels=1, **kw) == E["WORKSPACE"]
    # Ozaki leaves need their slice workspace; unsupported slice counts are
    # rejected before any device work
    assert _call(lib, base=1, **kw) == E["WORKSPACE"]
    assert _call(lib, base=1, slices=24 if P == 2 else 20, **kw) == E["UNSUPPORTED"]


def test_last_error_message(lib):
    assert _call(lib, lda=1) == E["ARG"]
    assert b"ld of A" in lib.ddqd_last_error()


def test_workspace_queries(lib):
    assert lib.dd_gemm_workspace(128, 128, 128, 1, 0, 0, 0) == 0
    one = lib.dd_gemm_workspace(128, 128, 128, 3, 1, 0, 0)
    # one level: 7 left operands, 7 right operands, 7 products of 64x64 DD
    assert one >= 7 * 3 * 64 * 64 * 16
    two = lib.dd_gemm_workspace(128, 128, 128, 3, 2, 0, 0)
    assert two > one
    q = lib.qd_gemm_workspace(128, 128, 128, 3, 1, 0, 0)
    assert q >= 2 * (one - 1024)
    assert lib.dd_gemm_workspace(-1, 1, 1, 1, 0, 0, 0) == ctypes.c_size_t(-1).value
    # depth stops when a dimension would drop below 2
    assert lib.dd_gemm_workspace(3, 64, 64, 2, 5, 0, 0) == lib.dd_gemm_workspace(3, 64, 64, 2, 1, 0, 0)


def test_empty_problems_are_no_ops(lib):
    # m == 0 or n == 0 returns before any device work, even without a GPU
    assert _call(lib, m=0) == E["OK"]
    assert _call(lib, n=0, fn="qd_gemm") == E["OK"]


@pytest.mark.skipif(on_gpu(), reason="checks the no-device path")
def test_valid_call_without_device_reports_nodevice(lib):
    assert _call(lib) == E["NODEVICE"]


def test_lu_argument_errors(lib):
    import ctypes as C
    A, ip, info = 0x10000, 0x40000, 0x50000
    # n, A, lda, psa, ipiv, perm, info, panel, pivot, algo, levels, base, ws, ws_bytes, stream
    lib.dd_getrf.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                             C.c_size_t, C.c_void_p]
    ok = dict(n=8, A=A, lda=8, psa=64, ipiv=ip, perm=None, info=info, panel=4, pivot=1, algo=1,
              levels=0, base=0, ws=None, wsb=0)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.dd_getrf(a["n"], a["A"], a["lda"], a["psa"], a["ipiv"], a["perm"], a["info"],
                            a["panel"], a["pivot"], a["algo"], a["levels"], a["base"], a["ws"],
                            a["wsb"], None)
    assert call(n=-1) == E["ARG"]
    assert call(panel=-2) == E["ARG"]
    assert call(panel=-1) == E["NODEVICE"]      # DDQD_PANEL_AUTO: a valid width
    # panel 0 is the row-wise comparator: no pivoting, no workspace
    assert call(panel=0) == E["UNSUPPORTED"]
    assert lib.dd_getrf_workspace(1024, 0, 3, 2, 1) == 0
    assert call(pivot=3) == E["ARG"]
    assert call(info=None) == E["ARG"]
    assert call(lda=4) == E["ARG"]
    assert call(n=9000, lda=9000, psa=9000 * 9000) == E["UNSUPPORTED"]
    assert call(algo=3, levels=2) == E["WORKSPACE"]
    assert lib.dd_getrf_workspace(1024, 128, 1, 0, 0) == 0
    assert lib.dd_getrf_workspace(1024, 128, 3, 1, 0) > 0
    lib.dd_getrs.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_size_t,
                             C.c_void_p]
    # B overlapping LU
    assert lib.dd_getrs(8, 2, A, 8, 64, ip, None, A + 16, 2, 16, 0x90000, 1 << 20,
                        None) == E["ALIAS"]
    assert lib.dd_getrs(8, 2, A, 8, 64, None, None, 0x70000, 2, 16, 0x90000, 1 << 20,
                        None) == E["ARG"]
    assert lib.dd_getrs(8, 2, A, 8, 64, ip, None, 0x70000, 2, 16, None, 0, None) == E["WORKSPACE"]
    assert lib.dd_getrs(0, 2, A, 8, 64, ip, None, 0x70000, 2, 16, None, 0, None) == E["OK"]


def test_graph_argument_errors(lib):
    import ctypes as C
    h = C.c_void_p(0x1234)
    assert lib.ddqd_graph_begin(None) == E["ARG"]
    assert lib.ddqd_graph_end(None, C.byref(h)) == E["ARG"]
    assert h.value is None                      # cleared on every error path
    assert lib.ddqd_graph_end(C.c_void_p(0x1000), None) == E["ARG"]
    assert lib.ddqd_graph_launch(None, None) == E["ARG"]
    assert lib.ddqd_graph_destroy(None) == E["OK"]


def test_tune_defaults_and_errors(lib):
    from paper_1510_08642_amd import ddqd
    ddqd.tune_clear()
    d = ddqd.tune_lookup(2, 1024, 1024, 1024)
    assert (d["algo"], d["levels"], d["tile"], d["candidates"]) == ("block", 0, 64, 0)
    assert ddqd.tune_lookup(2, 100, 100, 100)["tile"] == 32        # 64x64 tiles would idle CUs
    assert ddqd.tune_lookup(2, 100, 100, 100, base="ozaki")["tile"] == 0
    q = ddqd.tune_lookup(4, 1024, 1024, 1024)
    assert (q["algo"], q["levels"]) == ("winograd", 3)
    assert ddqd.tune_lookup(4, 200, 200, 200)["algo"] == "block"
    assert ddqd.tune_lookup(4, 200, 200, 200)["tile"] == 16       # 32x32 tiles would idle CUs
    assert ddqd.tune_lookup(4, 2048, 2048, 2048)["tile"] == 32
    assert ddqd.tune_lookup(2, 1024, 1024, 1024, base="ozaki")["band"] == 0
    import ctypes as C
    r = ddqd.TuneResult()
    assert lib.ddqd_tune_lookup(3, 8, 8, 8, 0, 0, C.byref(r)) == E["ARG"]
    assert lib.ddqd_tune_lookup(4, 8, 8, 8, 3, 0, C.byref(r)) == E["ARG"]
    assert ddqd.tune_lookup(4, 1024, 1024, 1024, base="crt")["algo"] == "block"
    assert ddqd.tune_lookup(4, 1024, 1024, 1024, base="ozaki")["algo"] == "block"
    assert lib.ddqd_tune_lookup(2, 8, 8, 8, 0, 0, None) == E["ARG"]
    # reps out of range is rejected before any device work
    assert lib.dd_gemm_tune(8, 8, 8, 0x10000, 8, 64, 0x20000, 8, 64, 0x30000, 8, 64, 0, 0, 0,
                            None, 0, None, None) == E["ARG"]


def test_lu_panel_tuner_defaults_workspace_and_errors(lib):
    import ctypes as C
    from paper_1510_08642_amd import ddqd
    ddqd.tune_clear()
    for P in (2, 4):
        d = ddqd.getrf_panel_lookup(P, 2048, algo="winograd", levels=1, base="ozaki")
        assert d == dict(panel=128, candidates=0, ms=0.0)
    # the AUTO workspace covers every width the tuner may choose (K = 32 .. 320)
    for P, f in ((2, lib.dd_getrf_workspace), (4, lib.qd_getrf_workspace)):
        for n in (40, 300, 2048):
            auto = f(n, -1, 3, 1, 1)
            assert auto != ddqd.SIZE_MAX
            for K in [32 * a for a in range(1, 11) if 32 * a <= n] + [128]:
                assert auto >= f(n, K, 3, 1, 1), (P, n, K)
        assert f(64, -2, 1, 0, 0) == ddqd.SIZE_MAX
    # tuning workspace: a copy of A, the pivots, and the product workspace
    tw = lib.ddqd_getrf_tune_workspace(2, 300, 3, 1, 1)
    assert tw >= 2 * 300 * 300 * 8 + 4 * 601 + lib.dd_getrf_workspace(300, -1, 3, 1, 1)
    assert lib.ddqd_getrf_tune_workspace(3, 300, 3, 1, 1) == ddqd.SIZE_MAX
    assert lib.ddqd_getrf_tune_workspace(2, 9000, 3, 1, 1) == ddqd.SIZE_MAX
    panel, cands, ms = C.c_int(0), C.c_int(0), C.c_double(0.0)
    assert lib.ddqd_getrf_panel_lookup(3, 64, 1, 1, 0, 0, C.byref(panel), None, None) == E["ARG"]
    assert lib.ddqd_getrf_panel_lookup(2, 64, 2, 1, 0, 0, C.byref(panel), None, None) == E["ARG"]
    assert lib.ddqd_getrf_panel_lookup(2, 64, 1, 1, 0, 0, None, None, None) == E["ARG"]
    assert lib.ddqd_getrf_panel_lookup(2, 64, 1, 1, 0, 0, C.byref(panel), C.byref(cands),
                                       C.byref(ms)) == E["OK"]
    assert (panel.value, cands.value) == (128, 0)
    # argument errors before any device work
    A = 0x10000
    assert lib.ddqd_getrf_tune(3, 8, A, 8, 64, 1, 1, 0, 0, 1, 0x90000, 1 << 20, None, None,
                               None) == E["ARG"]
    assert lib.ddqd_getrf_tune(2, 8, A, 8, 64, 1, 1, 0, 0, 0, 0x90000, 1 << 20, None, None,
                               None) == E["ARG"]
    assert lib.ddqd_getrf_tune(2, 8, A, 4, 64, 1, 1, 0, 0, 1, 0x90000, 1 << 20, None, None,
                               None) == E["ARG"]
    assert lib.ddqd_getrf_tune(2, 8, A, 8, 64, 1, 1, 0, 0, 1, None, 0, None, None,
                               None) == E["WORKSPACE"]
    assert lib.ddqd_getrf_tune(2, 8, A, 8, 64, 1, 1, 0, 0, 1, 0x90000, 1 << 20, None, None,
                               None) == E["NODEVICE"]


def test_latency_probe_argument_errors(lib):
    import ctypes as C
    out = C.c_void_p(0x10000)
    assert lib.ddqd_latency_probe(None, 64, 16, None) == E["ARG"]
    assert lib.ddqd_latency_probe(out, 128, 16, None) == E["ARG"]
    assert lib.ddqd_latency_probe(out, 64, 0, None) == E["ARG"]
    assert lib.ddqd_latency_probe(out, 64, 16, None) == E["NODEVICE"]


def test_auto_workspace_covers_every_candidate(lib):
    for P, f in ((2, lib.dd_gemm_workspace), (4, lib.qd_gemm_workspace)):
        for (m, n, l) in [(1024, 1024, 1024), (300, 129, 257), (40, 40, 40)]:
            auto = f(m, n, l, 4, 0, 0, 0)
            for algo, levels in [(1, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)]:
                if min(m, n, l) >> levels >= 16 or levels == 0:
                    assert auto >= f(m, n, l, algo, levels, 0, 0)
    o = lib.dd_gemm_workspace(512, 512, 512, 4, 0, 1, 0)
    assert o >= lib.dd_gemm_workspace(512, 512, 512, 3, 3, 1, 0)
    qo = lib.qd_gemm_workspace(512, 512, 512, 4, 0, 1, 0)
    assert qo >= lib.qd_gemm_workspace(512, 512, 512, 3, 3, 1, 0)


def test_qd_ozaki_workspace(lib):
    """QD Ozaki leaves: S INT8 slices of A and B in 32x32 fragment blocks
    plus the row / column exponents; slice counts outside 28..31 give none."""
    n = 256
    ws = lib.qd_gemm_workspace(n, n, n, 1, 0, 1, 0)
    assert ws >= 2 * 31 * n * n + 4 * 2 * n
    assert lib.qd_gemm_workspace(n, n, n, 1, 0, 1, 28) < ws
    assert lib.qd_gemm_workspace(n, n, n, 1, 0, 1, 20) == 0
    assert lib.qd_gemm_workspace(n, n, n, 1, 0, 1, 16) == 0


def test_qd_lu_argument_errors(lib):
    import ctypes as C
    from paper_1510_08642_amd import ddqd  # noqa: F401  (sets argtypes)
    A, ip, info = 0x10000, 0x40000, 0x50000
    call = lambda base, n=8, lda=8: lib.qd_getrf(n, A, lda, lda * n, ip, None, info, 4, 1, 1, 0,
                                                 base, None, 0, None)
    assert call(0, lda=4) == E["ARG"]
    assert call(3) == E["ARG"]
    assert lib.qd_getrf_workspace(64, 16, 3, 1, 3) == C.c_size_t(-1).value
    # QD trailing updates may run on Ozaki leaves (31 slices by default) or
    # on the CRT base
    assert lib.qd_getrf_workspace(1024, 128, 3, 1, 1) > lib.qd_getrf_workspace(1024, 128, 3, 1, 0)
    assert lib.qd_getrf_workspace(1024, 128, 3, 1, 2) > lib.qd_getrf_workspace(1024, 128, 3, 1, 0)
    assert lib.qd_getrs_workspace(100, 3) >= 4 * 8 * 100 * 3
    assert lib.qd_getrs_workspace(100, 3) > lib.dd_getrs_workspace(100, 3)


def test_getrs_noalloc_argument_errors(lib):
    f = lib.dd_getrs_noalloc
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    assert f(-1, 1, 0x10000, 4, 16, 0x20000, None, 0x30000, 1, 4, None) == E["ARG"]
    assert f(0, 1, None, 1, 1, None, None, None, 1, 1, None) == E["OK"]
    assert f(5, 0, None, 1, 1, None, None, None, 1, 1, None) == E["OK"]
    # orders beyond the fixed buffer are refused before any device call
    assert f(8193, 1, 0x10000, 8193, 8193 * 8193, 0x20000, None, 0x30000, 1, 8193,
             None) == E["UNSUPPORTED"]
    assert b"scratch limit" in lib.ddqd_last_error()


def test_grouped_descriptor_errors_and_workspace(lib):
    from paper_1510_08642_amd import ddqd
    D = ddqd.GemmDesc
    lib.dd_gemm_grouped_workspace.argtypes = [ctypes.c_int, ctypes.POINTER(D)]
    lib.dd_gemm_grouped_workspace.restype = ctypes.c_size_t
    lib.dd_gemm_grouped.argtypes = [ctypes.c_int, ctypes.POINTER(D), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]
    SIZE_MAX = ctypes.c_size_t(-1).value

    def desc(base=0, slices=0, m=64, n=64, l=64, A=0x100000, B=0x200000, C=0x300000):
        return D(m, n, l, 1, 0, base, slices, A, l, m * l, B, n, l * n, C, n, m * n)
    arr = (D * 2)(desc(), desc(base=1, A=0x400000, B=0x500000, C=0x600000))
    # FMA problems need no workspace; an Ozaki one needs its slices
    assert lib.dd_gemm_grouped_workspace(1, arr) == 0
    need = lib.dd_gemm_grouped_workspace(2, arr)
    assert need >= 2 * 16 * 64 * 64
    assert lib.dd_gemm_grouped(2, arr, None, 0, None) == E["WORKSPACE"]
    bad = (D * 1)(desc(base=3))
    assert lib.dd_gemm_grouped_workspace(1, bad) == SIZE_MAX
    assert lib.dd_gemm_grouped(1, bad, None, 0, None) == E["ARG"]
    bad = (D * 1)(desc(base=1, slices=30))
    assert lib.dd_gemm_grouped(1, bad, None, 0, None) == E["UNSUPPORTED"]
    # an output overlapping another problem's input
    alias = (D * 2)(desc(), desc(A=0x300000 + 64, C=0x700000))
    assert lib.dd_gemm_grouped(2, alias, None, 0, None) == E["ALIAS"]
    assert lib.dd_gemm_grouped(0, None, None, 0, None) == E["OK"]
    assert lib.dd_gemm_grouped(-1, None, None, 0, None) == E["ARG"]


def test_crt_moduli_cover_the_product_range(lib):
    """The CRT base's moduli for K = l: pairwise coprime, each fits INT8
    residues (<= 256), and their product M exceeds 2 kc 2^214 (kc = min(l,
    65536)), so the rebuilt integer product, |X| <= kc (2^107)^2, is unique."""
    import math
    from paper_1510_08642_amd import ddqd
    for l, want in [(1, 29), (32, 29), (1024, 30), (2048, 30), (4096, 31), (65536, 31),
                    (1 << 20, 31)]:
        ms = ddqd.crt_moduli(l)
        assert len(ms) == want, (l, ms)
        assert all(2 <= m <= 256 for m in ms)
        assert all(math.gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])
        M = math.prod(ms)
        kc = min(l, 65536)
        assert M > 2 * kc * 2 ** 214
        # the set is minimal for this rule: one modulus fewer does not cover it
        assert math.log2(math.prod(ms[:-1])) < math.log2(2 * kc * 2 ** 214) + 0.01
    assert lib.ddqd_crt_moduli(2, 0, None, 0) == -1
    assert lib.ddqd_crt_moduli(3, 64, None, 0) == -1
    assert lib.ddqd_crt_moduli(2, 64, None, -1) == -1


def test_crt_qd_moduli_cover_the_cross_term(lib):
    """QD: the 214-bit integers split as T = H 2^108 + L with |H| <= 2^106 and
    |L| <= 2^107 (1 + 2^-35); the larger of the two exact products is the
    cross term, |sum_k H_a L_b + L_a H_b| <= kc 2^214 (1 + 2^-35) (kc =
    min(l, 32768), the cross product running over 2 kc), so M must exceed
    twice that; both products share the set."""
    import math
    from paper_1510_08642_amd import ddqd
    for l, want in [(1, 29), (33, 29), (34, 30), (1024, 30), (2048, 30), (3835, 30),
                    (3836, 31), (32768, 31), (1 << 20, 31)]:
        ms = ddqd.crt_moduli(l, precision=4)
        assert len(ms) == want, (l, ms)
        assert all(math.gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])
        kc = min(l, 32768)
        M = math.prod(ms)
        # 2 kc 2^214 (1 + 2^-35) < M, in exact integers
        assert 2 * kc * (2 ** 249 + 2 ** 214) < M * 2 ** 35
        assert math.log2(math.prod(ms[:-1])) < 215 + math.log2(kc) + 0.01
    assert ddqd.crt_moduli(1024, precision=2) == ddqd.crt_moduli(1024)


def test_crt_base_arguments(lib):
    # the CRT base takes no slice count; QD runs it (the workspace is checked
    # before any device work)
    assert _call(lib, fn="qd_gemm", base=2) == E["WORKSPACE"]
    assert _call(lib, fn="qd_gemm", base=2, slices=30) == E["ARG"]
    assert _call(lib, base=2, slices=16) == E["ARG"]
    assert _call(lib, base=3) == E["ARG"]
    lib.dd_gemm_workspace.restype = ctypes.c_size_t
    lib.qd_gemm_workspace.restype = ctypes.c_size_t
    SIZE_MAX = 2 ** 64 - 1
    # n = 1024: 30 moduli of 1 KB fragments for A, B and C, plus exponents
    w = lib.dd_gemm_workspace(1024, 1024, 1024, 1, 0, 2, 0)
    assert 3 * 30 * 1024 * 1024 <= w < 3 * 30 * 1024 * 1024 + (1 << 20)
    # QD, n = 1024: 30 moduli; H and L residues of A and B (2 KB a line's
    # 32-block) and two products' residues of C
    w = lib.qd_gemm_workspace(1024, 1024, 1024, 1, 0, 2, 0)
    assert 6 * 30 * 1024 * 1024 <= w < 6 * 30 * 1024 * 1024 + (1 << 20)
    assert lib.dd_gemm_workspace(64, 64, 64, 1, 0, 2, 8) == SIZE_MAX
