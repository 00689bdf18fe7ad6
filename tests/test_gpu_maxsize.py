"""GPU parity at the largest transform lengths the library accepts
(N <= 2^24): m = 2 products whose d_H fills N = 2^24 (a power of two),
N = 3 * 2^22 (the longest odd-factor length below the limit) and N = 5 * 2^21
(the longest factor-5 length, three-pass with 2048-point rows; complex128,
which has no factor-5 kernels, takes 3 * 2^22 there), in complex64 and
complex128, on inputs shaped like the large single product (h an 8-term
exponential sum plus CN(0, 1e-6) noise, x ~ CN(0, 1/n)).  Sampled outputs y_i
are compared with the oracle's direct sums on exactly the inputs the GPU sees;
the scalar alpha = x^T H x is compared with sum_i x_i y_i over the call's own
full output (an identity of the order-2 product that holds at any size).  Tolerances: relative 2-norm error
<= 1e-12 (FP64) / 1e-4 (FP32)."""
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

# (n, expected transform length): d_H = 2n - 1
CASES = [((1 << 23), 1 << 24), (3 << 21, 3 << 22), (5 << 20, 5 << 21)]


@functools.lru_cache(maxsize=None)
def inputs(n):
    g = wl.rng_for(91, n)
    h, _ = wl.exp_sum_vector(g, 2 * n - 1, 8, 1e-3)
    return h, wl.cn(g, n, 1.0 / n)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n,n_fft", CASES)
def test_longest_transforms(dtype, n, n_fft):
    import paper_1401_6238_amd as hk
    d_h = 2 * n - 1
    if dtype == torch.complex64:
        assert hk.hk_fft_layout(d_h)[0] == n_fft
    print_case(test="maxsize", dtype=dtype, n=n, N=n_fft)
    h, x = inputs(n)
    hd, xd = to_dev(h, dtype), to_dev(x, dtype)
    y, a = hk.hankel_tvp(hd, xd, 2, True, True)
    torch.cuda.synchronize()
    hs, xs = seen(h, dtype), seen(x, dtype)
    del hd
    idx = np.unique(np.concatenate([np.arange(48), np.arange(n - 48, n),
                                    np.random.default_rng(n).integers(0, n, 64)]))
    yo, _ = oracle.tvp_sampled(2, [n, n], hs, [xs, xs], idx)
    yg = host(y)
    assert rel(yg[idx], yo) <= TOL[dtype]
    # alpha = x^T (H x) over the whole output, summed in FP64 on the host
    check_alpha(complex(host(a.reshape(1))[0]), complex(np.dot(xs, yg)), dtype)
