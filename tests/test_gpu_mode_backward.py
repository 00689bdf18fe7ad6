"""GPU adjoint of the products with distinct vectors, 1D (hankel_mode_products)
and BHHB (block_hankel_tvp), against the oracle's direct-sum gradients
(oracle.mode_backward / oracle.block_backward, pinned on the CPU by torch
autograd through dense tensors), through the C ABI and through the autograd
Functions; resident and three-pass layouts, non-square dims (n_p != N_p for
BHHB), both cotangents, one of them, and partial gradient requests.
Tolerance: relative 2-norm error <= 1e-12 (FP64) / 1e-4 (FP32) per gradient."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402

DTYPES = [torch.complex128, torch.complex64]


def draw(seed, dims, block_dims=None, scale_x=None):
    g = wl.rng_for(77, seed)
    m = len(dims)
    lens = [dims[p] * (block_dims[p] if block_dims else 1) for p in range(m)]
    hl = sum(dims) - m + 1
    if block_dims:
        hl *= sum(block_dims) - m + 1
    h = wl.cn(g, hl, 1.0)
    xs = [wl.cn(g, n, 1.0 / n if scale_x is None else scale_x) for n in lens]
    v = wl.cn(g, lens[0], 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    return h, xs, v, phi


def check_grads(gv, gh, ov, oh, dtype, want=None):
    tol = TOL[dtype]
    for p, (a, b) in enumerate(zip(gv, ov)):
        if want is not None and not want[p]:
            assert a is None
            continue
        if np.abs(b).max() == 0.0:
            assert np.abs(host(a)).max() == 0.0, p
        else:
            assert rel(host(a), b) <= tol, (p, rel(host(a), b))
    if gh is not None:
        assert rel(host(gh), oh) <= tol


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dims", [(300, 500), (64, 80, 50), (3000, 2000, 4000), (1200, 900, 1500, 700)])
@pytest.mark.parametrize("cot", ["both", "v", "phi"])
def test_mode_backward_vs_oracle(dtype, dims, cot):
    import paper_1401_6238_amd as hk
    m = len(dims)
    print_case(test="mode_backward", dtype=dtype, dims=dims, cot=cot)
    h, xs, v, phi = draw(sum(dims), dims)
    v = v if cot != "phi" else None
    phi = phi if cot != "v" else None
    hd = to_dev(h, dtype)
    xd = [to_dev(x, dtype) for x in xs]
    vd = to_dev(v, dtype) if v is not None else None
    pd = to_dev(np.array([phi]), dtype) if phi is not None else None
    gv, gh = hk.hankel_mode_products_backward(hd, xd, dims, vd, pd)
    torch.cuda.synchronize()
    ov, oh = oracle.mode_backward(m, dims, seen(h, dtype), [seen(x, dtype) for x in xs],
                                  seen(v, dtype) if v is not None else None,
                                  complex(seen(np.array([phi]), dtype)[0]) if phi is not None else None)
    check_grads(gv, gh, ov, oh, dtype)


@pytest.mark.parametrize("want,want_h", [((False, True, False), False), ((True, False, False), True),
                                         ((False, False, True), False)])
def test_mode_backward_partial(want, want_h):
    import paper_1401_6238_amd as hk
    dims = (2500, 3100, 1900)
    dtype = torch.complex128
    h, xs, v, phi = draw(5, dims)
    gv, gh = hk.hankel_mode_products_backward(to_dev(h, dtype), [to_dev(x, dtype) for x in xs], dims,
                                              to_dev(v, dtype), to_dev(np.array([phi]), dtype), want, want_h)
    ov, oh = oracle.mode_backward(3, dims, h, xs, v, phi)
    assert (gh is None) == (not want_h)
    check_grads(gv, gh, ov, oh, dtype, want)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dims,bdims", [((30, 20), (25, 15)), ((20, 24, 18), (16, 12, 22)), ((9, 7, 5, 6), (5, 8, 6, 4))])
@pytest.mark.parametrize("cot", ["both", "v", "phi"])
def test_block_backward_vs_oracle(dtype, dims, bdims, cot):
    import paper_1401_6238_amd as hk
    m = len(dims)
    print_case(test="block_backward", dtype=dtype, dims=dims, bdims=bdims, cot=cot)
    H, xs, v, phi = draw(sum(dims) + 7 * sum(bdims), dims, bdims, scale_x=0.3)
    v = v if cot != "phi" else None
    phi = phi if cot != "v" else None
    Hd = to_dev(H, dtype)
    xd = [to_dev(x, dtype) for x in xs]
    gv, gH = hk.block_hankel_tvp_backward(Hd, xd, dims, bdims, to_dev(v, dtype) if v is not None else None,
                                          to_dev(np.array([phi]), dtype) if phi is not None else None)
    torch.cuda.synchronize()
    ov, oH = oracle.block_backward(m, dims, bdims, seen(H, dtype), [seen(x, dtype) for x in xs],
                                   seen(v, dtype) if v is not None else None,
                                   complex(seen(np.array([phi]), dtype)[0]) if phi is not None else None)
    check_grads(gv, gH, ov, oH, dtype)


def test_mode_products_autograd():
    """The autograd Function: loss Re<w, y> + Re(conj(psi) alpha) with lazily
    conjugated cotangents; gradients of h and every vector against the oracle."""
    import paper_1401_6238_amd as hk
    dims = (2200, 1700, 2600)
    dt = torch.complex128
    h, xs, w, psi = draw(9, dims)
    ht = to_dev(h, dt).requires_grad_(True)
    xt = [to_dev(x, dt).requires_grad_(True) for x in xs]
    y, a = hk.hankel_mode_products_autograd(ht, xt, dims)
    loss = (y.conj() * to_dev(w, dt)).real.sum() + (a.conj() * torch.tensor(psi, dtype=dt, device=ht.device)).real
    grads = torch.autograd.grad(loss, [ht] + xt)
    ov, oh = oracle.mode_backward(3, dims, h, xs, w, psi)
    assert rel(host(grads[0]), oh) <= TOL[dt]
    for p in range(3):
        assert rel(host(grads[1 + p]), ov[p]) <= TOL[dt]


def test_block_autograd():
    import paper_1401_6238_amd as hk
    dims, bdims = (20, 24, 18), (16, 12, 22)
    dt = torch.complex128
    H, xs, w, psi = draw(10, dims, bdims, scale_x=0.3)
    Ht = to_dev(H, dt).requires_grad_(True)
    xt = [to_dev(x, dt).requires_grad_(True) for x in xs]
    y, a = hk.block_hankel_tvp_autograd(Ht, xt, dims, bdims)
    gr = torch.autograd.grad([y, a], [Ht] + xt, [to_dev(w, dt), torch.tensor(psi, dtype=dt, device=Ht.device)])
    ov, oH = oracle.block_backward(3, dims, bdims, H, xs, w, psi)
    assert rel(host(gr[0]), oH) <= TOL[dt]
    for p in range(3):
        assert rel(host(gr[1 + p]), ov[p]) <= TOL[dt]


def test_equal_vectors_through_distinct_adjoint():
    """One tensor passed for every mode: the distinct-vector gradients add up
    to the equal-vector adjoint (hankel_tvp_backward), both on the GPU, and
    match the oracle's equal-vector gradient."""
    import paper_1401_6238_amd as hk
    m, n = 4, 2000
    dt = torch.complex128
    h, xs, v, phi = draw(11, (n,) * m)
    x = xs[1]
    hd, xd, vd, pd = to_dev(h, dt), to_dev(x, dt), to_dev(v, dt), to_dev(np.array([phi]), dt)
    gv, gh = hk.hankel_mode_products_backward(hd, [xd] * m, [n] * m, vd, pd)
    gx_eq, gh_eq = hk.hankel_tvp_backward(hd, xd, m, vd, pd)
    ox, oh = oracle.tvp_backward(m, h, x, v, phi)
    total = sum(host(g) for g in gv)
    assert rel(total, ox) <= TOL[dt] and rel(host(gh), oh) <= TOL[dt]
    assert rel(total, host(gx_eq)) <= TOL[dt] and rel(host(gh), host(gh_eq)) <= TOL[dt]


@pytest.fixture
def smallest_lengths():
    """Odd-factor lengths for every size (the 'smallest' length policy)."""
    import paper_1401_6238_amd as hk
    hk.hk_set_fft_lengths("smallest")
    yield
    hk.hk_set_fft_lengths("auto")


# (dims, N for complex64): resident 3 * 64 and 5 * 1024, three-pass 3 * 8192
ODD_1D = [((64, 80, 50), 192), ((1200, 900, 1500, 700), 5120), ((9000, 8000, 7002), 24576)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dims,n_fft", ODD_1D)
def test_mode_backward_odd_lengths(smallest_lengths, dtype, dims, n_fft):
    """The distinct-vector adjoint on transform lengths 3 * 2^k and 5 * 2^k:
    its conjugating and generating-vector-free forward programs run on the
    odd-factor rows (resident and three-pass); every gradient against the
    oracle."""
    import paper_1401_6238_amd as hk
    m = len(dims)
    if dtype == torch.complex64:
        assert hk.hk_fft_layout(sum(dims) - m + 1)[0] == n_fft
    print_case(test="mode_backward_odd", dtype=dtype, dims=dims)
    h, xs, v, phi = draw(3 * sum(dims), dims)
    gv, gh = hk.hankel_mode_products_backward(to_dev(h, dtype), [to_dev(x, dtype) for x in xs], dims,
                                              to_dev(v, dtype), to_dev(np.array([phi]), dtype))
    torch.cuda.synchronize()
    ov, oh = oracle.mode_backward(m, dims, seen(h, dtype), [seen(x, dtype) for x in xs], seen(v, dtype),
                                  complex(seen(np.array([phi]), dtype)[0]))
    check_grads(gv, gh, ov, oh, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cot", ["both", "phi"])
def test_block_backward_odd_grid(smallest_lengths, dtype, cot):
    """The BHHB adjoint on a grid of 3 x 64 rows and 5 x 64 columns (n_p != N_p)
    against the oracle."""
    import paper_1401_6238_amd as hk
    dims, bdims = (70, 60, 62), (100, 100, 102)
    assert hk.block_hankel_tvp_layout(dtype, 3, dims, bdims, 1) == (192, 320)
    print_case(test="block_backward_odd", dtype=dtype, cot=cot)
    H, xs, v, phi = draw(911, dims, bdims, scale_x=0.3)
    v = v if cot != "phi" else None
    gv, gH = hk.block_hankel_tvp_backward(to_dev(H, dtype), [to_dev(x, dtype) for x in xs], dims, bdims,
                                          to_dev(v, dtype) if v is not None else None,
                                          to_dev(np.array([phi]), dtype))
    torch.cuda.synchronize()
    ov, oH = oracle.block_backward(3, dims, bdims, seen(H, dtype), [seen(x, dtype) for x in xs],
                                   seen(v, dtype) if v is not None else None,
                                   complex(seen(np.array([phi]), dtype)[0]))
    check_grads(gv, gH, ov, oH, dtype)
