"""Shared helpers for the tests: device transfer and error measures."""
from __future__ import annotations

import numpy as np

import oracle

U = 2.0 ** -53


def on_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def to_dev(X: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


def to_host(T) -> np.ndarray:
    return T.detach().cpu().numpy()


def rownorm_den(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """max_j (|A||B|)_ij per row i, from the leading components."""
    return (np.abs(A[0]) @ np.abs(B[0])).max(axis=1)


def rownorm_error(A, B, C, ii, jj, alpha=1, C0=None, den=None):
    """max over samples of |C_ij - E_ij| / max_j (|A||B|)_ij, E exact."""
    err = np.abs(oracle.exact_error(A, B, C, ii, jj, alpha=alpha, C0=C0))
    if den is None:
        den = rownorm_den(A, B)
        if C0 is not None:
            den = np.maximum(den, np.abs(C0[0]).max(axis=1))
    return float(np.max(err / den[ii]))


def all_entries(m, n):
    return np.repeat(np.arange(m), n), np.tile(np.arange(n), m)


def sample_entries(m, n, count, seed=0):
    g = np.random.default_rng(seed)
    ii = np.concatenate([[0, m - 1, 0, m - 1], g.integers(0, m, count)])
    jj = np.concatenate([[0, n - 1, n - 1, 0], g.integers(0, n, count)])
    return ii, jj


def value_diff(X, Y):
    """|X - Y| as values (component sums), elementwise, in float64 (enough to
    compare two results that agree to far more than 53 bits: the difference is
    formed component-wise before rounding)."""
    d = np.zeros(X.shape[1:])
    for c in range(max(X.shape[0], Y.shape[0])):
        xc = X[c] if c < X.shape[0] else 0.0
        yc = Y[c] if c < Y.shape[0] else 0.0
        d = d + (xc - yc)
    return np.abs(d)
