"""CPU oracle for DD/QD matrix products and DD LU (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never calls it, and the two
share no code: this is plain C compiled with gcc (``liboracle.so``), written
from the paper's definitions and from published error-free arithmetic.

Numbers are held in *plane layout*: a DD matrix is a float64 array of shape
``(2, rows, cols)`` (hi plane, lo plane), a QD matrix ``(4, rows, cols)``.

What each routine follows (paper: Kouya, arXiv 1510.08642):
  * ``gemm``: Simple (Sec. 2, Eq. 1), Block (Sec. 2), Strassen / Winograd with
    a recursion depth (Sec. 2; the textbook formulas, the paper's figures
    being unavailable), in the oracle's DD or QD arithmetic.
  * ``exact_entries`` / ``exact_error``: Eq. 1 evaluated exactly as a
    floating-point expansion, rounded once (the measurement reference).
  * ``getrf`` / ``getrs``: the blocked LU of Sec. 4 (steps 1-3), with optional
    partial pivoting, and the triangular solves of Eq. 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ALGOS = {"simple": 0, "block": 1, "strassen": 2, "winograd": 3}

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compiles liboracle.so with the Makefile beside this file."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-C", _HERE, "-B" if force else "liboracle.so"],
                       check=True, capture_output=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, c_int = ctypes.c_int64, ctypes.c_int
        L.or_gemm.argtypes = [c_int, c_int, c_int, c_int, i64, i64, i64, _D, _D, _D]
        L.or_gemm.restype = c_int
        L.or_exact_entries.argtypes = [c_int, i64, i64, i64, c_int, c_int, _D, _D, _D, i64,
                                       _I64, _I64, c_int, _D]
        L.or_exact_error.argtypes = [c_int, i64, i64, i64, c_int, c_int, _D, _D, _D, i64,
                                     _I64, _I64, c_int, _D, _D]
        L.or_exact_dot_expansion.argtypes = [c_int, i64, _D, i64, _D, i64, _D, c_int]
        L.or_exact_dot_expansion.restype = c_int
        L.or_expansion_sum.argtypes = [_D, c_int, _D]
        L.or_expansion_sum.restype = c_int
        L.or_expansion_round.argtypes = [_D, c_int, c_int, _D]
        L.or_elementwise.argtypes = [c_int, c_int, i64, _D, _D, _D]
        L.or_eft.argtypes = [c_int, i64, _D, _D, _D, _D]
        L.or_getrf.argtypes = [i64, _D, _I32, c_int, c_int, c_int, c_int, c_int]
        L.or_getrf.restype = c_int
        L.or_getrs.argtypes = [i64, i64, _D, _I32, _D]
        L.or_getrs.restype = c_int
        L.or_getrf_p.argtypes = [c_int, i64, _D, _I32, c_int, c_int, c_int, c_int, c_int]
        L.or_getrf_p.restype = c_int
        L.or_getrs_p.argtypes = [c_int, i64, i64, _D, _I32, _D]
        L.or_getrs_p.restype = c_int
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = c_int
        L.or_set_threads.argtypes = [c_int]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def gemm(A: np.ndarray, B: np.ndarray, algo: str = "block", levels: int = 0,
         bs: int = 32) -> np.ndarray:
    """C := A B in the oracle's DD (P=2) or QD (P=4) arithmetic."""
    A, B = _f64(A), _f64(B)
    P, m, l = A.shape
    P2, l2, n = B.shape
    assert P == P2 and l == l2 and P in (2, 4)
    C = np.zeros((P, m, n))
    rc = lib().or_gemm(P, ALGOS[algo], levels, bs, m, n, l, _dp(A), _dp(B), _dp(C))
    if rc:
        raise ValueError("or_gemm rejected its arguments")
    return C


def _samples(ii, jj):
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    assert ii.shape == jj.shape and ii.ndim == 1
    return ii, jj


def exact_entries(A, B, ii, jj, kout: int = 4, alpha: int = 1, C0=None) -> np.ndarray:
    """Exact alpha*(A B)_ij (+ C0_ij) at the samples, rounded to kout terms.

    C0, if given, is the full matrix in plane layout (beta = 1).  Returns an
    array of shape (kout, nsamples)."""
    A, B = _f64(A), _f64(B)
    P, m, l = A.shape
    n = B.shape[2]
    ii, jj = _samples(ii, jj)
    c0 = None
    if C0 is not None:
        C0 = _f64(C0)
        c0 = _f64(np.concatenate([C0[:P, ii, jj],
                                  np.zeros((max(0, P - C0.shape[0]), len(ii)))]))
    out = np.zeros((kout, len(ii)))
    lib().or_exact_entries(P, m, n, l, alpha, 0 if C0 is None else 1, _dp(A), _dp(B),
                           _dp(c0) if c0 is not None else None, len(ii),
                           ii.ctypes.data_as(_I64), jj.ctypes.data_as(_I64), kout, _dp(out))
    return out


def exact_error(A, B, Chat, ii, jj, alpha: int = 1, C0=None) -> np.ndarray:
    """(exact alpha*(A B) + C0) - Chat at the samples, as doubles.

    Chat is the computed matrix in plane layout with any number of planes,
    or, if 2-D, its values at the samples already gathered (planes, nsamples)."""
    A, B = _f64(A), _f64(B)
    P, m, l = A.shape
    n = B.shape[2]
    ii, jj = _samples(ii, jj)
    Chat = np.asarray(Chat)
    ch = _f64(Chat if Chat.ndim == 2 else Chat[:, ii, jj])
    c0 = None
    if C0 is not None:
        C0 = _f64(C0)
        c0 = _f64(np.concatenate([C0[:P, ii, jj],
                                  np.zeros((max(0, P - C0.shape[0]), len(ii)))]))
    err = np.zeros(len(ii))
    lib().or_exact_error(P, m, n, l, alpha, 0 if C0 is None else 1, _dp(A), _dp(B),
                         _dp(c0) if c0 is not None else None, len(ii),
                         ii.ctypes.data_as(_I64), jj.ctypes.data_as(_I64), ch.shape[0],
                         _dp(ch), _dp(err))
    return err


def exact_dot_expansion(x: np.ndarray, y: np.ndarray, cap: int = 4096) -> np.ndarray:
    """The exact expansion of sum_k x_k y_k for (P, l) vectors."""
    x, y = _f64(x), _f64(y)
    P, l = x.shape
    out = np.zeros(cap)
    k = lib().or_exact_dot_expansion(P, l, _dp(x), l, _dp(y), l, _dp(out), cap)
    if k < 0:
        raise ValueError("expansion longer than cap")
    return out[:k].copy()


def expansion_sum(vals) -> np.ndarray:
    v = _f64(vals)
    out = np.zeros(len(v) + 1)
    k = lib().or_expansion_sum(_dp(v), len(v), _dp(out))
    return out[:k].copy()


def expansion_round(vals, k: int) -> np.ndarray:
    v = _f64(vals)
    out = np.zeros(k)
    lib().or_expansion_round(_dp(v), len(v), k, _dp(out))
    return out


_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3}


def elementwise(op: str, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """z = x op y on (cnt, P) arrays of DD (P=2) or QD (P=4) numbers."""
    x, y = _f64(x), _f64(y)
    cnt, P = x.shape
    z = np.zeros_like(x)
    lib().or_elementwise(P, _OPS[op], cnt, _dp(x), _dp(y), _dp(z))
    return z


def eft(op: str, a, b):
    """('two_sum' | 'fast_two_sum' | 'two_prod') over arrays -> (s, e)."""
    a, b = _f64(a), _f64(b)
    s, e = np.zeros_like(a), np.zeros_like(a)
    lib().or_eft({"two_sum": 0, "fast_two_sum": 1, "two_prod": 2}[op], a.size, _dp(a), _dp(b),
                 _dp(s), _dp(e))
    return s, e


def getrf(A: np.ndarray, panel: int = 64, pivot: bool = True, algo: str = "winograd",
          levels: int = 1, bs: int = 32):
    """Blocked LU in DD (A of shape (2, n, n)) or QD ((4, n, n)).  Returns
    (LU in plane layout, ipiv int32, info)."""
    LU = _f64(A).copy()
    P, n = LU.shape[0], LU.shape[1]
    ipiv = np.zeros(n, dtype=np.int32)
    info = lib().or_getrf_p(P, n, _dp(LU), ipiv.ctypes.data_as(_I32), panel, int(pivot),
                            ALGOS[algo], levels, bs)
    if info < 0:
        raise ValueError("or_getrf_p rejected its arguments")
    return LU, ipiv, info


def getrs(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solves A X = B from getrf's factors; B is (P, n, nrhs) like LU."""
    LU = _f64(LU)
    X = _f64(B).copy()
    P, n, nrhs = X.shape[0], X.shape[1], X.shape[2]
    assert LU.shape[0] == P
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    if lib().or_getrs_p(P, n, nrhs, _dp(LU), ipiv.ctypes.data_as(_I32), _dp(X)) < 0:
        raise ValueError("or_getrs_p rejected its arguments")
    return X


def lu_residual(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> float:
    """max_j ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf), the residual formed
    exactly (one rounding at the end)."""
    A = _f64(A)
    n = A.shape[1]
    nrhs = X.shape[2]
    ii = np.repeat(np.arange(n), nrhs)
    jj = np.tile(np.arange(nrhs), n)
    r = exact_entries(A, X, ii, jj, kout=1, alpha=-1, C0=B)[0].reshape(n, nrhs)
    normA = np.max(np.sum(np.abs(A[0]), axis=1))
    normx = np.max(np.abs(X[0]), axis=0)
    return float(np.max(np.max(np.abs(r), axis=0) / (normA * normx)))


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return lib().or_num_threads()


def set_threads(t: int) -> None:
    lib().or_set_threads(t)
