"""dd_getrs_noalloc (the solve with the library's fixed per-GPU buffer in
place of a workspace), called through the C ABI: bit-identical to dd_getrs
with its own workspace, on two calls in a row, the second on a smaller
system (the buffer keeps the first call's contents), with and without the
permutation vector, and with more than 16 right-hand sides (two passes through
the buffer)."""
import ctypes

import numpy as np
import pytest

from paper_1510_08642_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


def factored(dd, n, seed):
    import torch
    g = inputs.rng(seed)
    A = torch.from_numpy(inputs.dd_lu_matrix(n, g, boost=False)).cuda()
    ipiv, perm, info = dd.dd_getrf(A, panel=64, algo="block", levels=0)
    B = torch.from_numpy(inputs.dd_uniform(n, 24, g)).cuda()
    return A, ipiv, perm, B


def noalloc_call(dd, LU, ipiv, perm, X):
    """The C-ABI call itself (ctypes), on torch's current stream."""
    import torch
    n, nrhs = X.shape[1], X.shape[2]
    lib = dd.lib()
    st = lib.dd_getrs_noalloc(n, nrhs, LU.data_ptr(), LU.stride(1), LU.stride(0),
                              ipiv.data_ptr() if ipiv is not None else None,
                              perm.data_ptr() if perm is not None else None,
                              X.data_ptr(), X.stride(1), X.stride(0),
                              torch.cuda.current_stream().cuda_stream)
    assert st == 0, lib.ddqd_last_error()


@pytest.mark.parametrize("use_perm", [True, False])
def test_noalloc_solve_matches_getrs(dd, use_perm):
    import torch
    for n, nrhs in ((1500, 20), (333, 3)):          # the second call is smaller
        print(f"case getrs_noalloc n={n} nrhs={nrhs} perm={use_perm}", flush=True)
        LU, ipiv, perm, B = factored(dd, n, 900 + n)
        p = perm if use_perm else None
        ref = B[:, :, :nrhs].contiguous()
        dd.dd_getrs(LU, ipiv, ref, perm=p)
        X = B[:, :, :nrhs].contiguous()
        noalloc_call(dd, LU, ipiv, p, X)
        torch.cuda.synchronize()
        assert torch.equal(X, ref), (n, nrhs)


def test_noalloc_rejects_orders_above_its_buffer(dd):
    import torch
    lib = dd.lib()
    X = torch.zeros((2, 1, 1), dtype=torch.float64, device="cuda")
    st = lib.dd_getrs_noalloc(8193, 1, X.data_ptr(), 8193, 8193 * 8193, None, X.data_ptr(),
                              X.data_ptr(), 1, 8193, None)
    assert st == 4 and b"scratch limit" in lib.ddqd_last_error()
