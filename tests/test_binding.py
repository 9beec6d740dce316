"""The Python binding's own argument checks, without a GPU.

The C ABI sees pointers, leading dimensions and plane strides only, so a view
whose shape does not match the problem (a row slice of a larger tensor given
as C, an LU factor of the wrong order, a short pivot vector) would pass its
stride checks and be written beyond its storage.  The binding must reject such
arguments by shape before anything reaches the library."""
import pytest
import torch

from paper_1510_08642_amd import ddqd


def dd(*shape):
    return torch.zeros((2,) + shape, dtype=torch.float64)


@pytest.mark.parametrize("fn,P", [(ddqd.dd_gemm, 2), (ddqd.qd_gemm, 4)])
def test_gemm_rejects_output_of_wrong_shape(fn, P):
    A = torch.zeros((P, 100, 100), dtype=torch.float64)
    B = torch.zeros((P, 100, 100), dtype=torch.float64)
    big = torch.zeros((P, 100, 100), dtype=torch.float64)
    # rows 60.. of a 100 x 100 matrix: ld and plane stride look valid for a
    # 100 x 100 C, but only 40 rows exist
    with pytest.raises(ValueError, match="C must have shape"):
        fn(A, B, big[:, 60:, :])
    # extra columns: would be written only in part
    with pytest.raises(ValueError, match="C must have shape"):
        fn(A, B, torch.zeros((P, 100, 120), dtype=torch.float64))
    with pytest.raises(ValueError, match="C must have shape"):
        fn(A, B, torch.zeros((2 if P == 4 else 4, 100, 100), dtype=torch.float64))


def test_gemm_rejects_inner_mismatch_and_bad_rank():
    with pytest.raises(ValueError):
        ddqd.dd_gemm(dd(4, 5), dd(6, 4))
    with pytest.raises(ValueError):
        ddqd.dd_gemm(torch.zeros((4, 5), dtype=torch.float64), dd(5, 4))


@pytest.mark.parametrize("fn,P", [(ddqd.dd_getrs, 2), (ddqd.qd_getrs, 4)])
def test_getrs_checks_factor_and_pivot_sizes(fn, P):
    n = 16
    B = torch.zeros((P, n, 3), dtype=torch.float64)
    ipiv = torch.zeros(n, dtype=torch.int32)
    LU = torch.zeros((P, n, n), dtype=torch.float64)
    with pytest.raises(ValueError, match="LU must have shape"):
        fn(torch.zeros((P, n - 1, n - 1), dtype=torch.float64), ipiv, B)
    with pytest.raises(ValueError, match="LU must have shape"):
        fn(torch.zeros((P, 2 * n, 2 * n), dtype=torch.float64)[:, 1:, :], ipiv, B)
    with pytest.raises(ValueError, match="ipiv"):
        fn(LU, ipiv[: n - 1], B)
    with pytest.raises(ValueError, match="ipiv"):
        fn(LU, ipiv.to(torch.int64), B)
    with pytest.raises(ValueError, match="perm"):
        fn(LU, ipiv, B, perm=torch.zeros(n - 2, dtype=torch.int32))
    with pytest.raises(ValueError, match="both None"):
        fn(LU, None, B)


def test_getrf_requires_square():
    with pytest.raises(ValueError, match="square"):
        ddqd.dd_getrf(dd(8, 9))
