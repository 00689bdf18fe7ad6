"""GPU parity of the transform lengths 3 * 2^k and 5 * 2^k against the CPU
oracle.  Such a length is computed as a 2D transform of 3 or 5 power-of-two
sequences through the Chinese-remainder index map; these cases pin every
layout the planner picks for it (resident and 3-pass, each odd factor, both
precisions, the degenerate one-element sequences), distinct-vector and scalar
products, the float adjoint, strided batches, grouped plans that mix odd and
power-of-two lengths (also against a power-of-two-only plan of the same
problems) and tensor-matrix products.  Tolerances as in the other parity
tests: relative 2-norm error <= 1e-12 in FP64, <= 1e-4 in FP32."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, oracle_problem, print_case, rel, seen, to_dev  # noqa: E402
from test_gpu_batched import check_plan_outputs, mixed_problems, plan_inputs  # noqa: E402
from test_gpu_parity import check  # noqa: E402


@pytest.fixture(autouse=True, scope="module")
def smallest_lengths():
    """These tests pin the odd-factor kernels, so every call here takes the
    smallest length (the default policy takes them for large work only)."""
    import paper_1401_6238_amd as hk
    hk.hk_set_fft_lengths("smallest")
    yield
    hk.hk_set_fft_lengths("auto")


def layout(d):
    """(odd factor, multipass) of the complex64 layout of d_H = d."""
    import paper_1401_6238_amd as hk
    n, r, c = hk.hk_fft_layout(d)
    return n // (r * c), c > 1


# (m, n, odd factor, multipass) of the complex64 layout of d_H = m (n - 1) + 1
FWD_CASES = [(2, 2, 3, False), (2, 3, 5, False), (3, 64, 3, False), (3, 700, 5, False), (3, 1000, 3, False),
             (4, 1365, 3, False), (3, 4096, 3, True), (3, 6000, 5, True), (4, 2731, 3, True),
             (5, 4096, 5, True), (2, 40000, 5, True)]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128, torch.float32, torch.float64])
@pytest.mark.parametrize("m,n,odd,multi", FWD_CASES)
def test_forward_equal(dtype, m, n, odd, multi):
    assert layout(m * (n - 1) + 1) == (odd, multi)
    print_case(test="odd_forward_equal", dtype=dtype, m=m, n=n, odd=odd)
    prob = wl.random_problem(9100 + 7 * m + n, m, [n] * m, True, complex_=dtype.is_complex, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("dims,odd,multi", [([700, 500, 900], 5, False), ([3, 3, 1], 5, False),
                                            ([4000, 3000, 5284], 3, True), ([2000, 3000, 2500, 4000], 3, True),
                                            ([9000, 8000], 5, True)])
def test_forward_distinct(dtype, dims, odd, multi):
    m = len(dims)
    assert layout(sum(dims) - m + 1) == (odd, multi)
    print_case(test="odd_forward_distinct", dtype=dtype, dims=dims)
    prob = wl.random_problem(9200 + sum(dims), m, dims, False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("m,n", [(3, 1000), (3, 4096), (4, 2731), (2, 2)])
def test_backward(dtype, m, n):
    """complex64 adjoints of these shapes run on odd lengths; complex128 ones
    keep power-of-two lengths (same oracle, same bar)."""
    import paper_1401_6238_amd as hk
    print_case(test="odd_backward", dtype=dtype, m=m, n=n)
    g = wl.rng_for(41, m * 100000 + n)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    gx, gh = hk.hankel_tvp_backward(to_dev(h, dtype), to_dev(x, dtype), m, to_dev(v, dtype),
                                    to_dev(np.array([phi]), dtype))
    torch.cuda.synchronize()
    ox, oh = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), seen(v, dtype),
                                 complex(seen(np.array([phi]), dtype)[0]))
    assert rel(host(gx), ox) <= TOL[dtype]
    assert rel(host(gh), oh) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("m,n,B", [(3, 700, 5), (3, 4096, 3), (5, 4096, 2)])
def test_strided_batched(dtype, m, n, B):
    import paper_1401_6238_amd as hk
    print_case(test="odd_strided", dtype=dtype, m=m, n=n, B=B)
    probs = [wl.random_problem(9300 + b, m, [n] * m, True, complex_=True, want_alpha=True) for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        yo, ao = oracle_problem(p, dtype)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        check_alpha(complex(host(a[b:b + 1])[0]), ao, dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_plan_odd_and_pow2(dtype):
    """A grouped plan of mixed sizes (odd and power-of-two lengths, resident
    and 3-pass) against the oracle, and the same plan restricted to
    power-of-two lengths against the oracle too."""
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    print_case(test="odd_plan", dtype=dtype)
    probs = mixed_problems(35, 60)
    for extra, (m, n) in enumerate([(3, 4096), (3, 6000), (4, 2731), (3, 700)]):
        probs.append(wl.random_problem(9400 + extra, m, [n] * m, True, want_alpha=True))
    odd = sum(1 for p in probs if not p.is_block and layout(sum(p.dims) - p.m + 1)[0] > 1)
    assert odd >= 20
    plan = hk.Plan(plan_inputs(probs, dtype))
    outs = plan.execute()
    plan.status()
    check_plan_outputs(probs, outs, dtype)
    plan2 = hk.Plan(plan_inputs(probs, dtype), flags=_lib.HK_PLAN_POW2)
    outs2 = plan2.execute()
    plan2.status()
    check_plan_outputs(probs, outs2, dtype)
    plan.close()
    plan2.close()


@pytest.mark.parametrize("m,n,R", [(3, 700, 2), (3, 4096, 3), (4, 1365, 2)])
def test_tensor_matrix(m, n, R):
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    print_case(test="odd_tensor_matrix", m=m, n=n, R=R)
    g = wl.rng_for(42, m * 1000 + n)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    U = wl.cn(g, n * R, 1.0 / n).reshape(n, R)
    T = hk.hankel_tensor_matrix(to_dev(h, dtype), to_dev(U, dtype), m)
    torch.cuda.synchronize()
    To = oracle.tensor_matrix(m, seen(h, dtype), seen(U, dtype))
    assert rel(host(T), To) <= TOL[dtype]


def test_factor5_threepass_under_default_policy():
    """Under the default policy a strided batch with instances * N >= 2^22
    takes the three-pass length 5 * 2^14 (d_H = 71,998 < 81,920): its result
    is bit-identical to the smallest-length policy's (same length, same
    kernels) and matches the oracle on sampled instances."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    m, n, B = 3, 24000, 64
    probs = [wl.random_problem(6100 + b, m, [n] * m, True, want_alpha=True) for b in (0, 31, 63)]
    g = torch.Generator().manual_seed(61)
    H = (torch.randn(B, m * (n - 1) + 1, generator=g, dtype=torch.float64) / 2 ** 0.5).to(dtype)
    X = (torch.randn(B, n, generator=g, dtype=torch.float64) / (2 * n) ** 0.5).to(dtype)
    for k, b in enumerate((0, 31, 63)):
        H[b] = torch.from_numpy(probs[k].h).to(dtype)
        X[b] = torch.from_numpy(probs[k].vectors[1]).to(dtype)
    H, X = H.to("cuda"), X.to("cuda")
    print_case(test="factor5_threepass_auto", m=m, n=n, B=B)
    ys, a_s = hk.hankel_tvp_strided_batched(H, X, m, True, True)  # module policy: smallest
    hk.hk_set_fft_lengths("auto")
    try:
        ya, aa = hk.hankel_tvp_strided_batched(H, X, m, True, True)
        hk.hk_set_fft_lengths("pow2")
        yp, _ = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    finally:
        hk.hk_set_fft_lengths("smallest")
    torch.cuda.synchronize()
    assert torch.equal(ya, ys) and torch.equal(aa, a_s)
    assert not torch.equal(ya, yp)
    for k, b in enumerate((0, 31, 63)):
        p = probs[k]
        yo, ao = oracle.tvp(m, [n] * m, seen(p.h, dtype), [seen(p.vectors[1], dtype)] * m, True, True)
        assert rel(host(ya[b]), yo) <= TOL[dtype], b
        check_alpha(complex(host(aa[b:b + 1])[0]), ao, dtype, b)
