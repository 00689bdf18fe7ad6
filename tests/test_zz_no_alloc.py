"""hankel_tvp_noalloc (static device workspace) against hankel_tvp (caller
workspace) through the C ABI: two calls in a row on one device, the second
with a smaller input, so that the second runs on what the first left in the
shared array.  Both entry points run the same kernels with the same schedule,
so the results agree bit for bit; the relative 2-norm error bound of the
products (1e-12 FP64, 1e-4 FP32) is checked as well, and the small products
against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

HK_DT = {torch.complex64: 0, torch.complex128: 1, torch.float32: 2, torch.float64: 3}


def _noalloc(h, x, m):
    """y = H x^{m-1}, alpha = H x^m through the C ABI entry point."""
    from paper_1401_6238_amd._lib import check, lib
    n = x.numel()
    y = torch.empty(n, dtype=x.dtype, device=x.device)
    a = torch.empty(1, dtype=x.dtype, device=x.device)
    st = torch.cuda.current_stream(x.device).cuda_stream
    check(lib().hankel_tvp_noalloc(HK_DT[x.dtype], h.data_ptr(), m, n, x.data_ptr(), y.data_ptr(), a.data_ptr(),
                                   ctypes.c_void_p(st)), "hankel_tvp_noalloc")
    return y, a


def _case(seed, m, n, dtype):
    prob = wl.random_problem(seed, m, [n] * m, True, complex_=dtype.is_complex, want_alpha=True)
    return prob, to_dev(prob.h, dtype), to_dev(prob.vectors[1], dtype)


def _compare(m, h, x, dtype):
    import paper_1401_6238_amd as hk
    y0, a0 = hk.hankel_tvp(h, x, m, True, True)
    y1, a1 = _noalloc(h, x, m)
    torch.cuda.synchronize()
    Y0, Y1 = host(y0), host(y1)
    A0, A1 = complex(host(a0.reshape(1))[0]), complex(host(a1)[0])
    assert rel(Y1, Y0) <= TOL[dtype]
    check_alpha(A1, A0, dtype, "no-alloc vs hankel_tvp")
    assert np.array_equal(Y1, Y0) and A1 == A0, "same kernels and schedule: results must agree bit for bit"
    return Y1, A1


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_noalloc_two_calls_second_smaller(dtype):
    # first: the large single product's shape (m = 4, n = 2^18, N = 2^20, three passes)
    print_case(test="noalloc", dtype=dtype, m=4, n=1 << 18)
    p = wl.large_single(0)
    h = to_dev(p.h, dtype)
    x = to_dev(p.vectors[1], dtype)
    _compare(4, h, x, dtype)
    del h, x
    # second, smaller (three passes on a shorter grid, then resident), each also against the oracle
    for seed, m, n in ((31, 3, 5000), (32, 3, 64)):
        print_case(test="noalloc", dtype=dtype, m=m, n=n)
        prob, h, x = _case(seed, m, n, dtype)
        y, a = _compare(m, h, x, dtype)
        yo, ao = oracle.tvp(m, prob.dims, seen(prob.h, dtype), [seen(v, dtype) for v in prob.vectors], True, True)
        assert rel(y, yo) <= TOL[dtype]
        check_alpha(a, ao, dtype, "no-alloc vs oracle")


def test_noalloc_real_and_rejection():
    """Real FP64 input (resident, no workspace), then a product whose workspace
    exceeds the static array: rejected before anything is enqueued, and the
    next call still works."""
    from paper_1401_6238_amd._lib import HankelError, lib
    print_case(test="noalloc_real", dtype="f64", m=3, n=64)
    prob = wl.small_real()
    h = to_dev(prob.h, torch.float64)
    x = to_dev(prob.vectors[1], torch.float64)
    y, a = _compare(3, h, x, torch.float64)
    yo, ao = oracle.tvp(3, prob.dims, prob.h, prob.vectors, True, True)
    assert rel(y, yo.real) <= TOL[torch.float64]
    check_alpha(a, ao.real, torch.float64)
    # complex128, m = 4, n = 2^19: N = 2^21, two 32 MiB buffers > 40 MiB
    n = 1 << 19
    hb = torch.zeros(4 * (n - 1) + 1, dtype=torch.complex128, device="cuda")
    xb = torch.zeros(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(HankelError) as ei:
        _noalloc(hb, xb, 4)
    assert ei.value.code == 4 and b"HK_NOALLOC_SCRATCH_BYTES" in lib().hk_last_error()
    del hb, xb
    print_case(test="noalloc_after_rejection", dtype="c64", m=3, n=5000)
    prob, h, x = _case(33, 3, 5000, torch.complex64)
    _compare(3, h, x, torch.complex64)
