"""Thin ctypes binding of libddqd.so over torch device tensors.

Argument marshalling only: every arithmetic step runs in the HIP library.
A DD matrix is a float64 tensor of shape ``(2, rows, cols)`` on a GPU (a QD
matrix ``(4, rows, cols)``) whose last dimension is contiguous; its row
stride is the leading dimension and its plane stride the plane stride of the
C ABI (include/ddqd.h).  Work is enqueued on torch's current stream of the
tensors' device; workspace comes from torch's caching allocator.

If the library has not been built this module raises on import: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddqd.so")

ALGO = {"simple": 0, "block": 1, "strassen": 2, "winograd": 3, "auto": 4}
ALGO_NAME = {v: k for k, v in ALGO.items()}
BASE = {"fma": 0, "ozaki": 1, "crt": 2}
PIVOT = {"none": 0, "partial": 1}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_1510_08642_amd.build` (no CPU fallback exists)")

_lib = ctypes.CDLL(LIB_PATH)
_i64, _int, _vp, _sz = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t

_GEMM_ARGS = [_i64, _i64, _i64, _int, _vp, _i64, _i64, _vp, _i64, _i64, _int, _vp, _i64, _i64,
              _int, _int, _int, _int, _vp, _sz, _vp]
for _name in ("dd_gemm", "qd_gemm"):
    getattr(_lib, _name).argtypes = _GEMM_ARGS
    getattr(_lib, _name).restype = _int
for _name in ("dd_gemm_workspace", "qd_gemm_workspace"):
    getattr(_lib, _name).argtypes = [_i64, _i64, _i64, _int, _int, _int, _int]
    getattr(_lib, _name).restype = _sz
for _p in ("dd", "qd"):
    getattr(_lib, f"{_p}_getrf_workspace").argtypes = [_i64, _int, _int, _int, _int]
    getattr(_lib, f"{_p}_getrf_workspace").restype = _sz
    getattr(_lib, f"{_p}_getrf").argtypes = [_i64, _vp, _i64, _i64, _vp, _vp, _vp, _int, _int,
                                             _int, _int, _int, _vp, _sz, _vp]
    getattr(_lib, f"{_p}_getrf").restype = _int
    getattr(_lib, f"{_p}_getrs_workspace").argtypes = [_i64, _i64]
    getattr(_lib, f"{_p}_getrs_workspace").restype = _sz
    getattr(_lib, f"{_p}_getrs").argtypes = [_i64, _i64, _vp, _i64, _i64, _vp, _vp, _vp, _i64,
                                             _i64, _vp, _sz, _vp]
    getattr(_lib, f"{_p}_getrs").restype = _int
_lib.dd_getrs_noalloc.argtypes = [_i64, _i64, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _vp]
_lib.dd_getrs_noalloc.restype = _int
_PREC = {2: "dd", 4: "qd"}


class GemmDesc(ctypes.Structure):
    """ddqd_gemm_desc of include/ddqd.h."""
    _fields_ = [("m", _i64), ("n", _i64), ("l", _i64), ("alpha", _int), ("beta", _int),
                ("base", _int), ("slices", _int),
                ("A", _vp), ("lda", _i64), ("psa", _i64), ("B", _vp), ("ldb", _i64),
                ("psb", _i64), ("C", _vp), ("ldc", _i64), ("psc", _i64)]


_lib.dd_gemm_grouped.argtypes = [_int, ctypes.POINTER(GemmDesc), _vp, _sz, _vp]
_lib.dd_gemm_grouped.restype = _int
_lib.dd_gemm_grouped_workspace.argtypes = [_int, ctypes.POINTER(GemmDesc)]
_lib.dd_gemm_grouped_workspace.restype = _sz
_lib.ddqd_profile_enable.argtypes = [_int]
_lib.ddqd_profile_enable.restype = None
_lib.ddqd_profile_reset.argtypes = []
_lib.ddqd_profile_reset.restype = None
_lib.ddqd_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(_i64)]
_lib.ddqd_profile_query.restype = _int
_lib.ddqd_status_string.argtypes = [_int]
_lib.ddqd_status_string.restype = ctypes.c_char_p
_lib.ddqd_last_error.argtypes = []
_lib.ddqd_last_error.restype = ctypes.c_char_p


class TuneResult(ctypes.Structure):
    """ddqd_tune_result of include/ddqd.h."""
    _fields_ = [("algo", _int), ("levels", _int), ("tile", _int), ("band", _int),
                ("candidates", _int), ("ms", ctypes.c_double)]


for _name in ("dd_gemm_tune", "qd_gemm_tune"):
    getattr(_lib, _name).argtypes = [_i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _i64, _vp,
                                     _i64, _i64, _int, _int, _int, _vp, _sz, _vp,
                                     ctypes.POINTER(TuneResult)]
    getattr(_lib, _name).restype = _int
_lib.ddqd_tune_lookup.argtypes = [_int, _i64, _i64, _i64, _int, _int, ctypes.POINTER(TuneResult)]
_lib.ddqd_tune_lookup.restype = _int
_lib.ddqd_tune_clear.argtypes = []
_lib.ddqd_tune_clear.restype = None
_lib.ddqd_getrf_tune.argtypes = [_int, _i64, _vp, _i64, _i64, _int, _int, _int, _int, _int, _vp,
                                 _sz, _vp, ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)]
_lib.ddqd_getrf_tune.restype = _int
_lib.ddqd_getrf_tune_workspace.argtypes = [_int, _i64, _int, _int, _int]
_lib.ddqd_getrf_tune_workspace.restype = _sz
_lib.ddqd_getrf_panel_lookup.argtypes = [_int, _i64, _int, _int, _int, _int, ctypes.POINTER(_int),
                                         ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)]
_lib.ddqd_getrf_panel_lookup.restype = _int
_lib.ddqd_crt_moduli.argtypes = [_int, _i64, ctypes.POINTER(_int), _int]
_lib.ddqd_crt_moduli.restype = _int
_lib.ddqd_latency_probe.argtypes = [_vp, _int, _int, _vp]
_lib.ddqd_latency_probe.restype = _int
_lib.ddqd_graph_begin.argtypes = [_vp]
_lib.ddqd_graph_begin.restype = _int
_lib.ddqd_graph_end.argtypes = [_vp, ctypes.POINTER(_vp)]
_lib.ddqd_graph_end.restype = _int
_lib.ddqd_graph_launch.argtypes = [_vp, _vp]
_lib.ddqd_graph_launch.restype = _int
_lib.ddqd_graph_destroy.argtypes = [_vp]
_lib.ddqd_graph_destroy.restype = _int

SIZE_MAX = ctypes.c_size_t(-1).value
PANEL_AUTO = -1     # DDQD_PANEL_AUTO


def _panel(panel):
    return PANEL_AUTO if panel == "auto" else int(panel)


class DDQDError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.ddqd_status_string(status).decode()
        detail = _lib.ddqd_last_error().decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))


def lib() -> ctypes.CDLL:
    return _lib


def _check(status: int, where: str) -> None:
    if status != 0:
        raise DDQDError(status, where)


def _mat(X: torch.Tensor, P: int, name: str):
    if X.dim() != 3 or X.shape[0] != P:
        raise ValueError(f"{name} must have shape ({P}, rows, cols)")
    if X.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if X.numel() == 0:          # empty: strides are meaningless and never used
        return X.data_ptr(), max(1, X.shape[2]), max(1, X.shape[1] * X.shape[2])
    if X.shape[2] > 1 and X.stride(2) != 1:
        raise ValueError(f"{name} must be contiguous along its last dimension")
    return X.data_ptr(), X.stride(1), X.stride(0)


def _stream_of(X: torch.Tensor):
    if X.device.type != "cuda":
        raise ValueError("tensors must be on a GPU")
    return torch.cuda.current_stream(X.device).cuda_stream


def gemm_workspace(P: int, m: int, n: int, l: int, algo="block", levels=0, base="fma",
                   slices=0) -> int:
    f = _lib.dd_gemm_workspace if P == 2 else _lib.qd_gemm_workspace
    ws = f(m, n, l, ALGO[algo], levels, BASE[base], slices)
    if ws == SIZE_MAX:
        raise ValueError("invalid gemm arguments")
    return ws


def _gemm(P, A, B, C, alpha, beta, algo, levels, base, slices, ws):
    if A.dim() != 3 or B.dim() != 3:
        raise ValueError(f"A and B must have shape ({P}, rows, cols)")
    m, l = A.shape[1], A.shape[2]
    n = B.shape[2]
    if B.shape[1] != l:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = torch.empty((P, m, n), dtype=torch.float64, device=A.device)
        beta = 0
    elif tuple(C.shape) != (P, m, n):
        # the C ABI sees only pointers and strides: a C of another shape would
        # be written only in part, or beyond its storage
        raise ValueError(f"C must have shape ({P}, {m}, {n}), got {tuple(C.shape)}")
    pa, lda, psa = _mat(A, P, "A")
    pb, ldb, psb = _mat(B, P, "B")
    pc, ldc, psc = _mat(C, P, "C")
    need = gemm_workspace(P, m, n, l, algo, levels, base, slices)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    f = _lib.dd_gemm if P == 2 else _lib.qd_gemm
    st = f(m, n, l, alpha, pa, lda, psa, pb, ldb, psb, beta, pc, ldc, psc, ALGO[algo], levels,
           BASE[base], slices, ws.data_ptr(), ws.numel(), _stream_of(C))
    _check(st, "dd_gemm" if P == 2 else "qd_gemm")
    return C


def dd_gemm(A, B, C=None, *, alpha=1, beta=0, algo="block", levels=0, base="fma", slices=0,
            ws=None):
    """C := beta*C + alpha*(A B) in double-double; returns C."""
    return _gemm(2, A, B, C, alpha, beta, algo, levels, base, slices, ws)


def qd_gemm(A, B, C=None, *, alpha=1, beta=0, algo="block", levels=0, base="fma", slices=0,
            ws=None):
    """C := beta*C + alpha*(A B) in quad-double; returns C.  base="ozaki" runs
    the leaves on INT8 matrix cores with `slices` digits (0 = 31); base="crt"
    by residues of 214-bit integers (split in halves) and the Chinese
    remainder theorem."""
    return _gemm(4, A, B, C, alpha, beta, algo, levels, base, slices, ws)


def crt_moduli(l: int, precision: int = 2) -> list:
    """The moduli base="crt" uses for a product with K = l in DD (precision
    2) or QD (4) (host only)."""
    out = (_int * 32)()
    N = _lib.ddqd_crt_moduli(precision, l, out, 32)
    if N < 0:
        raise ValueError("l must be positive and precision 2 or 4")
    return list(out[:N])


def getrf_workspace(n: int, panel=128, algo="winograd", levels=1, base="fma", P: int = 2) -> int:
    ws = getattr(_lib, f"{_PREC[P]}_getrf_workspace")(n, _panel(panel), ALGO[algo], levels,
                                                      BASE[base])
    if ws == SIZE_MAX:
        raise ValueError("invalid getrf arguments")
    return ws


def dd_getrf(A, *, panel=128, pivot="partial", algo="winograd", levels=1, base="fma",
             want_perm=True, ws=None, out=None):
    """In-place DD LU of the square (2, n, n) tensor A (blocked right-looking,
    panel width `panel`, trailing update by `algo`/`levels`/`base`; panel=0
    is the paper's row-wise parallel comparator, pivot="none" only;
    panel="auto" the width getrf_tune chose for this order, else 128).

    Returns (ipiv, perm, info) as device int32 tensors: LAPACK-style 0-based
    interchanges, the resulting row permutation (or None), and info (0, or the
    1-based column of the first exactly-zero pivot).  `out` may supply those
    three tensors (perm may be None), e.g. for a call recorded in a graph."""
    return _getrf(2, A, panel, pivot, algo, levels, base, want_perm, ws, out)


def qd_getrf(A, *, panel=128, pivot="partial", algo="winograd", levels=1, base="fma",
             want_perm=True, ws=None, out=None):
    """As dd_getrf for a QD (4, n, n) tensor."""
    return _getrf(4, A, panel, pivot, algo, levels, base, want_perm, ws, out)


def _getrf(P, A, panel, pivot, algo, levels, base, want_perm, ws, out):
    n = A.shape[1]
    if A.dim() != 3 or A.shape[2] != n:
        raise ValueError("A must be square")
    pa, lda, psa = _mat(A, P, "A")
    dev = A.device
    if out is not None:
        ipiv, perm, info = out
        if ipiv.numel() < n or info.numel() < 1 or (perm is not None and perm.numel() < n):
            raise ValueError("out tensors are too small")
        if any(t is not None and (t.dtype != torch.int32 or not t.is_contiguous())
               for t in (ipiv, perm, info)):
            raise TypeError("out tensors must be contiguous int32")
    else:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if want_perm else None
        info = torch.empty(1, dtype=torch.int32, device=dev)
    need = getrf_workspace(n, panel, algo, levels, base, P)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    st = getattr(_lib, f"{_PREC[P]}_getrf")(
        n, pa, lda, psa, ipiv.data_ptr(), perm.data_ptr() if perm is not None else None,
        info.data_ptr(), _panel(panel), PIVOT[pivot], ALGO[algo], levels, BASE[base], ws.data_ptr(),
        ws.numel(), _stream_of(A))
    _check(st, f"{_PREC[P]}_getrf")
    return ipiv[:n], (perm[:n] if perm is not None else None), info


def dd_getrs(LU, ipiv, B, *, perm=None, ws=None):
    """Solves A X = B in place on B (2, n, nrhs) from dd_getrf's factors."""
    return _getrs(2, LU, ipiv, B, perm, ws)


def qd_getrs(LU, ipiv, B, *, perm=None, ws=None):
    """Solves A X = B in place on B (4, n, nrhs) from qd_getrf's factors."""
    return _getrs(4, LU, ipiv, B, perm, ws)


def _getrs(P, LU, ipiv, B, perm, ws):
    n, nrhs = B.shape[1], B.shape[2]
    if tuple(LU.shape) != (P, n, n):
        raise ValueError(f"LU must have shape ({P}, {n}, {n}), got {tuple(LU.shape)}")
    for name, v in (("ipiv", ipiv), ("perm", perm)):
        if v is not None and (v.dtype != torch.int32 or not v.is_contiguous() or v.numel() < n):
            raise ValueError(f"{name} must be a contiguous int32 tensor of at least {n} entries")
    if ipiv is None and perm is None:
        raise ValueError("ipiv and perm are both None")
    pl, ldl, psl = _mat(LU, P, "LU")
    pb, ldb, psb = _mat(B, P, "B")
    need = getattr(_lib, f"{_PREC[P]}_getrs_workspace")(n, nrhs)
    if need == SIZE_MAX:
        raise ValueError("invalid getrs arguments")
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=B.device)
    st = getattr(_lib, f"{_PREC[P]}_getrs")(
        n, nrhs, pl, ldl, psl, ipiv.data_ptr() if ipiv is not None else None,
        perm.data_ptr() if perm is not None else None, pb, ldb, psb, ws.data_ptr(), ws.numel(),
        _stream_of(B))
    _check(st, f"{_PREC[P]}_getrs")
    return B


def dd_getrs_noalloc(LU, ipiv, B, *, perm=None):
    """As dd_getrs, with no workspace: the library's fixed per-GPU buffer
    (orders up to 8192).  Calls that overlap on one GPU race."""
    n, nrhs = B.shape[1], B.shape[2]
    if tuple(LU.shape) != (2, n, n):
        raise ValueError(f"LU must have shape (2, {n}, {n}), got {tuple(LU.shape)}")
    for name, v in (("ipiv", ipiv), ("perm", perm)):
        if v is not None and (v.dtype != torch.int32 or not v.is_contiguous() or v.numel() < n):
            raise ValueError(f"{name} must be a contiguous int32 tensor of at least {n} entries")
    if ipiv is None and perm is None:
        raise ValueError("ipiv and perm are both None")
    pl, ldl, psl = _mat(LU, 2, "LU")
    pb, ldb, psb = _mat(B, 2, "B")
    st = _lib.dd_getrs_noalloc(n, nrhs, pl, ldl, psl,
                               ipiv.data_ptr() if ipiv is not None else None,
                               perm.data_ptr() if perm is not None else None, pb, ldb, psb,
                               _stream_of(B))
    _check(st, "dd_getrs_noalloc")
    return B


def dd_gemm_grouped(problems, *, base="fma", slices=0, ws=None, stream_of=None):
    """Several unrelated DD products in grouped launches.

    problems: list of (A, B, C, alpha, beta) with C preallocated, or
    (A, B, C, alpha, beta, base, slices) to give a problem its own base.
    Each result is bit-identical to dd_gemm(A, B, C, algo="block", base=...,
    slices=...)."""
    if not problems:
        return
    arr = (GemmDesc * len(problems))()
    for i, pr in enumerate(problems):
        A, B, C, alpha, beta = pr[:5]
        pbase, psl = (pr[5], pr[6]) if len(pr) > 5 else (base, slices)
        pa, lda, psa = _mat(A, 2, "A")
        pb, ldb, psb = _mat(B, 2, "B")
        pc, ldc, psc = _mat(C, 2, "C")
        if A.shape[2] != B.shape[1] or C.shape[1] != A.shape[1] or C.shape[2] != B.shape[2]:
            raise ValueError(f"problem {i}: shapes do not match")
        arr[i] = GemmDesc(A.shape[1], B.shape[2], A.shape[2], alpha, beta, BASE[pbase], psl,
                          pa, lda, psa, pb, ldb, psb, pc, ldc, psc)
    need = _lib.dd_gemm_grouped_workspace(len(problems), arr)
    if need == SIZE_MAX:
        raise ValueError("invalid grouped gemm arguments")
    dev = problems[0][2].device
    if need > 0 and (ws is None or ws.numel() < need):
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st = _lib.dd_gemm_grouped(len(problems), arr, ws.data_ptr() if need > 0 else None,
                              ws.numel() if need > 0 else 0,
                              _stream_of(problems[0][2]) if stream_of is None else stream_of)
    _check(st, "dd_gemm_grouped")


def profile_enable(on: bool = True) -> None:
    """Per-kernel event timing inside the library (diagnostics)."""
    _lib.ddqd_profile_enable(1 if on else 0)


def profile_reset() -> None:
    _lib.ddqd_profile_reset()


def profile_query(substr: str | None = None):
    """(total milliseconds, launches) of kernels whose name contains substr."""
    ms, cnt = ctypes.c_double(0.0), _i64(0)
    _check(_lib.ddqd_profile_query(substr.encode() if substr else None, ctypes.byref(ms),
                                   ctypes.byref(cnt)), "ddqd_profile_query")
    return ms.value, cnt.value


class Graph:
    """A recorded sequence of library calls (ddqd_graph_*): replay() launches
    it again on a stream; every tensor the calls used must stay alive."""

    def __init__(self, handle):
        self._h = handle

    def replay(self, stream=None):
        if self._h is None:
            raise RuntimeError("graph was released")
        s = torch.cuda.current_stream().cuda_stream if stream is None else stream
        _check(_lib.ddqd_graph_launch(self._h, s), "ddqd_graph_launch")

    def release(self):
        if self._h is not None:
            _lib.ddqd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.release()


def capture(fn, stream):
    """Records the library calls fn() makes on `stream` (a torch.cuda.Stream,
    not the default stream) and returns them as a Graph.  fn must allocate
    nothing on the device (pass workspaces and outputs in)."""
    s = stream.cuda_stream
    _check(_lib.ddqd_graph_begin(s), "ddqd_graph_begin")
    try:
        with torch.cuda.stream(stream):
            fn()
    finally:
        h = _vp()
        st = _lib.ddqd_graph_end(s, ctypes.byref(h))
    _check(st, "ddqd_graph_end")
    return Graph(h.value)


def _tune_dict(r: TuneResult):
    return dict(algo=ALGO_NAME[r.algo], levels=r.levels, tile=r.tile, band=r.band,
                candidates=r.candidates, ms=r.ms)


def tune(A, B, C=None, *, base="fma", slices=0, reps=3, ws=None):
    """Times the candidate configurations of this product shape (dd_gemm_tune /
    qd_gemm_tune by the number of planes) and caches the fastest for
    algo="auto"; C receives A B.  Returns the chosen configuration."""
    P = A.shape[0]
    if P not in (2, 4):
        raise ValueError("A must have 2 (DD) or 4 (QD) planes")
    m, l, n = A.shape[1], A.shape[2], B.shape[2]
    if C is None:
        C = torch.empty((P, m, n), dtype=torch.float64, device=A.device)
    pa, lda, psa = _mat(A, P, "A")
    pb, ldb, psb = _mat(B, P, "B")
    pc, ldc, psc = _mat(C, P, "C")
    need = gemm_workspace(P, m, n, l, "auto", 0, base, slices)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    r = TuneResult()
    fn = _lib.dd_gemm_tune if P == 2 else _lib.qd_gemm_tune
    _check(fn(m, n, l, pa, lda, psa, pb, ldb, psb, pc, ldc, psc, BASE[base], slices, reps,
              ws.data_ptr(), ws.numel(), _stream_of(C), ctypes.byref(r)), "gemm_tune")
    return _tune_dict(r)


def tune_lookup(P: int, m: int, n: int, l: int, base="fma", slices=0):
    """The configuration algo="auto" uses for this shape."""
    r = TuneResult()
    _check(_lib.ddqd_tune_lookup(P, m, n, l, BASE[base], slices, ctypes.byref(r)),
           "ddqd_tune_lookup")
    return _tune_dict(r)


def tune_clear() -> None:
    _lib.ddqd_tune_clear()


def getrf_tune(A, *, pivot="partial", algo="winograd", levels=1, base="fma", reps=2, ws=None):
    """Times dd_getrf / qd_getrf (by the number of planes) of a copy of A
    with the panel widths K = 32, 64, ..., 320 (those <= n) and caches the
    fastest for panel="auto"; A is not modified.  Returns
    dict(panel, ms, candidates)."""
    P, n = A.shape[0], A.shape[1]
    if P not in (2, 4) or A.dim() != 3 or A.shape[2] != n:
        raise ValueError("A must be a square (2 | 4, n, n) tensor")
    pa, lda, psa = _mat(A, P, "A")
    need = _lib.ddqd_getrf_tune_workspace(P, n, ALGO[algo], levels, BASE[base])
    if need == SIZE_MAX:
        raise ValueError("invalid getrf_tune arguments")
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    panel, ms = _int(0), ctypes.c_double(0.0)
    _check(_lib.ddqd_getrf_tune(P, n, pa, lda, psa, PIVOT[pivot], ALGO[algo], levels, BASE[base],
                                reps, ws.data_ptr(), ws.numel(), _stream_of(A),
                                ctypes.byref(panel), ctypes.byref(ms)), "ddqd_getrf_tune")
    return getrf_panel_lookup(P, n, pivot=pivot, algo=algo, levels=levels, base=base)


def getrf_panel_lookup(P: int, n: int, *, pivot="partial", algo="winograd", levels=1,
                       base="fma"):
    """The panel width panel="auto" uses for this order and product."""
    panel, cands, ms = _int(0), _int(0), ctypes.c_double(0.0)
    _check(_lib.ddqd_getrf_panel_lookup(P, n, PIVOT[pivot], ALGO[algo], levels, BASE[base],
                                        ctypes.byref(panel), ctypes.byref(cands),
                                        ctypes.byref(ms)), "ddqd_getrf_panel_lookup")
    return dict(panel=panel.value, candidates=cands.value, ms=ms.value)


LATENCY_NAMES = ("fma", "add", "two_sum", "shuffle_max", "readlane2_add", "lds_roundtrip",
                 "two_barriers_lds", "fma_x4_independent")


def latency_probe(threads: int = 256, steps: int = 2048, device="cuda"):
    """ddqd_latency_probe: s_memtime ticks per dependent step of the LU column
    step's building blocks (a diagnostic; see include/ddqd.h)."""
    out = torch.zeros(9, dtype=torch.float64, device=device)
    s = torch.cuda.current_stream(out.device)
    _check(_lib.ddqd_latency_probe(out.data_ptr(), threads, steps, ctypes.c_void_p(s.cuda_stream)),
           "ddqd_latency_probe")
    s.synchronize()
    return dict(zip(LATENCY_NAMES, [round(v, 1) for v in out[:8].tolist()]))
