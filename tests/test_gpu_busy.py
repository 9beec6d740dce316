"""Products computed while another stream keeps the device busy.

Workgroups of a launch may then start long after one another; a kernel whose
workgroups read values that other workgroups of the same launch write would
give a different result than on a quiet device.  Every product path here must
give the quiet device's result bit for bit (the LU and its solve are checked
the same way in test_gpu_lu.py)."""
import pytest

from paper_1510_08642_amd import inputs
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available()
    from paper_1510_08642_amd import ddqd
    return ddqd


CASES = [(2, "block", 0, "fma"), (2, "winograd", 1, "fma"), (2, "block", 0, "ozaki"),
         (2, "strassen", 1, "ozaki"), (4, "block", 0, "fma"), (4, "winograd", 1, "fma"),
         (4, "block", 0, "ozaki"), (2, "block", 0, "crt"), (2, "winograd", 1, "crt")]


@pytest.mark.parametrize("P,algo,lv,base", CASES)
def test_products_with_the_device_busy_are_bit_identical(dd, P, algo, lv, base):
    import torch
    print(f"case busy P={P} {algo}{lv} {base}", flush=True)
    g = inputs.rng(31)
    gen = inputs.dd_uniform if P == 2 else inputs.qd_uniform
    m, n, l = 333, 290, 301
    A = to_dev(gen(m, l, g))
    B = to_dev(gen(l, n, g))
    prod = dd.dd_gemm if P == 2 else dd.qd_gemm
    ref = prod(A, B, algo=algo, levels=lv, base=base)
    torch.cuda.synchronize()
    big = 2048
    A2 = to_dev(inputs.dd_uniform(big, big, g))
    B2 = to_dev(inputs.dd_uniform(big, big, g))
    C2 = torch.empty_like(A2)
    ws2 = torch.empty(dd.gemm_workspace(2, big, big, big, "block", 0, "ozaki"),
                      dtype=torch.uint8, device=A2.device)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(4):
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s1):
            dd.dd_gemm(A2, B2, C2, base="ozaki", ws=ws2)
        with torch.cuda.stream(s2):
            C = prod(A, B, algo=algo, levels=lv, base=base)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), rep


def test_grouped_products_with_the_device_busy_are_bit_identical(dd):
    import torch
    print("case busy grouped", flush=True)
    g = inputs.rng(32)
    shapes = [(70, 40, 90), (128, 128, 128), (33, 257, 65), (200, 9, 120)]
    probs = []
    for (m, n, l) in shapes:
        probs.append((to_dev(inputs.dd_uniform(m, l, g)), to_dev(inputs.dd_uniform(l, n, g))))
    ref = [dd.dd_gemm(A, B, algo="block", base="fma") for A, B in probs]
    torch.cuda.synchronize()
    big = 2048
    A2 = to_dev(inputs.dd_uniform(big, big, g))
    B2 = to_dev(inputs.dd_uniform(big, big, g))
    C2 = torch.empty_like(A2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(4):
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s1):
            dd.dd_gemm(A2, B2, C2, base="ozaki")
        with torch.cuda.stream(s2):
            outs = [torch.empty((2, A.shape[1], B.shape[2]), dtype=torch.float64,
                                device=A.device) for A, B in probs]
            dd.dd_gemm_grouped([(A, B, C, 1, 0) for (A, B), C in zip(probs, outs)])
        torch.cuda.synchronize()
        for C, R in zip(outs, ref):
            assert torch.equal(C, R), rep
