"""GPU adjoint (J^H applied to cotangents) against the oracle's direct-sum
gradients, complex autograd through the Function wrapper, and the
dot-product identity evaluated entirely on the GPU."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402

DTYPES = [torch.complex128, torch.complex64]


def inputs(seed, m, n):
    g = wl.rng_for(40, seed)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    return h, x, v, phi


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n", [(2, 3), (3, 64), (4, 300), (5, 900), (3, 3000), (4, 2500), (2, 9000)])
@pytest.mark.parametrize("which", ["v", "phi", "both"])
def test_backward_vs_oracle(dtype, m, n, which):
    import paper_1401_6238_amd as hk
    print_case(test="backward", dtype=dtype, m=m, n=n, which=which)
    h, x, v, phi = inputs(m * 100000 + n, m, n)
    v = v if which != "phi" else None
    phi = phi if which != "v" else None
    hd, xd = to_dev(h, dtype), to_dev(x, dtype)
    vd = to_dev(v, dtype) if v is not None else None
    pd = to_dev(np.array([phi]), dtype) if phi is not None else None
    gx, gh = hk.hankel_tvp_backward(hd, xd, m, vd, pd)
    torch.cuda.synchronize()
    ox, oh = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), seen(v, dtype) if v is not None else None,
                                 complex(seen(np.array([phi]), dtype)[0]) if phi is not None else None)
    tol = TOL[dtype]
    assert rel(host(gx), ox) <= tol
    assert rel(host(gh), oh) <= tol


@pytest.mark.parametrize("want", [(True, False), (False, True)])
def test_backward_partial_outputs(want):
    import paper_1401_6238_amd as hk
    m, n = 4, 5000
    h, x, v, phi = inputs(7, m, n)
    dt = torch.complex128
    gx, gh = hk.hankel_tvp_backward(to_dev(h, dt), to_dev(x, dt), m, to_dev(v, dt), to_dev(np.array([phi]), dt),
                                    want_grad_x=want[0], want_grad_h=want[1])
    ox, oh = oracle.tvp_backward(m, h, x, v, phi)
    if want[0]:
        assert gh is None and rel(host(gx), ox) <= 1e-12
    else:
        assert gx is None and rel(host(gh), oh) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n,B", [(4, 200, 5), (3, 3000, 3)])
def test_backward_strided_batched(dtype, m, n, B):
    import paper_1401_6238_amd as hk
    print_case(test="backward_batched", dtype=dtype, m=m, n=n, B=B)
    data = [inputs(500 + b, m, n) for b in range(B)]
    H = torch.stack([to_dev(d[0], dtype) for d in data])
    X = torch.stack([to_dev(d[1], dtype) for d in data])
    V = torch.stack([to_dev(d[2], dtype) for d in data])
    P = to_dev(np.array([d[3] for d in data]), dtype)
    gx, gh = hk.hankel_tvp_backward_strided_batched(H, X, m, V, P)
    torch.cuda.synchronize()
    for b in range(B):
        h, x, v, phi = data[b]
        ox, oh = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), seen(v, dtype),
                                     complex(seen(np.array([phi]), dtype)[0]))
        assert rel(host(gx[b]), ox) <= TOL[dtype]
        assert rel(host(gh[b]), oh) <= TOL[dtype]


def test_autograd_matches_oracle():
    import paper_1401_6238_amd as hk
    m, n = 4, 3000
    h, x, v, phi = inputs(11, m, n)
    dt = torch.complex128
    ht = to_dev(h, dt).requires_grad_(True)
    xt = to_dev(x, dt).requires_grad_(True)
    g, f = hk.hankel_tvp_autograd(ht, xt, m)
    gx, gh = torch.autograd.grad([g, f], [xt, ht], [to_dev(v, dt), torch.tensor(phi, dtype=dt, device=ht.device)])
    ox, oh = oracle.tvp_backward(m, h, x, v, phi)
    assert rel(host(gx), ox) <= 1e-12
    assert rel(host(gh), oh) <= 1e-12


def test_autograd_gradcheck_tiny():
    import paper_1401_6238_amd as hk
    m, n = 3, 5
    h, x, _, _ = inputs(12, m, n)
    ht = to_dev(h, torch.complex128).requires_grad_(True)
    xt = to_dev(x, torch.complex128).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: hk.hankel_tvp_autograd(a, b, m), (ht, xt), eps=1e-6, atol=1e-8)


def test_dot_product_identity_on_gpu():
    """<v, J dx> = <J^H v, dx> with both sides computed by the GPU library."""
    import paper_1401_6238_amd as hk
    m, n = 4, 6000
    h, x, v, _ = inputs(13, m, n)
    dx = wl.cn(wl.rng_for(41, 0), n, 1.0)
    dt = torch.complex128
    hd, xd, vd, dxd = (to_dev(a, dt) for a in (h, x, v, dx))
    jdx, _ = hk.hankel_mode_products(hd, [None, dxd] + [xd] * (m - 2), [n] * m)
    gx, _ = hk.hankel_tvp_backward(hd, xd, m, vd, None, True, False)
    lhs = np.vdot(v, (m - 1) * host(jdx))
    rhs = np.vdot(host(gx), dx)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_backward_finite_differences_gpu():
    """Central differences (step 1e-6, FP64) of Re<v, g> + Re(conj(phi) f) through the GPU forward."""
    import paper_1401_6238_amd as hk
    m, n = 4, 400
    h, x, v, phi = inputs(14, m, n)
    dt = torch.complex128
    hd, xd = to_dev(h, dt), to_dev(x, dt)

    def loss(hh, xx):
        y, a = hk.hankel_tvp(to_dev(hh, dt), to_dev(xx, dt), m, True, True)
        return float(np.real(np.vdot(v, host(y))) + np.real(np.conj(phi) * complex(host(a.reshape(1))[0])))

    gx, gh = hk.hankel_tvp_backward(hd, xd, m, to_dev(v, dt), to_dev(np.array([phi]), dt))
    gx, gh = host(gx), host(gh)
    eps = 1e-6
    for l in [0, 123, n - 1]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            d = np.zeros(n, np.complex128)
            d[l] = eps * unit
            fd = (loss(h, x + d) - loss(h, x - d)) / (2 * eps)
            assert abs(fd - part(gx[l])) <= 1e-7 * max(1.0, abs(gx[l]))
    for s in [0, 777, len(h) - 1]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            d = np.zeros(len(h), np.complex128)
            d[s] = eps * unit
            fd = (loss(h + d, x) - loss(h - d, x)) / (2 * eps)
            assert abs(fd - part(gh[s])) <= 1e-7 * max(1.0, abs(gh[s]))


@pytest.mark.parametrize("batched", [False, True])
def test_autograd_conjugated_loss(batched):
    """Loss Re(sum conj(g) w) + Re(conj(f) psi): autograd hands the backward
    cotangents that can be lazy conjugate views; the gradients must still be
    J^H applied to (w, psi), the oracle's gradients."""
    import paper_1401_6238_amd as hk
    m, n, B = 3, 2000, (2 if batched else 1)
    dt = torch.complex128
    data = [inputs(60 + b, m, n) for b in range(B)]
    H = torch.stack([to_dev(d[0], dt) for d in data]).requires_grad_(True)
    X = torch.stack([to_dev(d[1], dt) for d in data]).requires_grad_(True)
    W = torch.stack([to_dev(d[2], dt) for d in data])
    psi = to_dev(np.array([d[3] for d in data]), dt)
    hh, xx = (H, X) if batched else (H[0], X[0])
    g, f = hk.hankel_tvp_autograd(hh, xx, m)
    ww, pp = (W, psi) if batched else (W[0], psi[0])
    loss = (g.conj() * ww).real.sum() + (f.conj() * pp).real.sum()
    gH, gX = torch.autograd.grad(loss, [H, X])
    for b, (h, x, w, ps) in enumerate(data):
        ox, oh = oracle.tvp_backward(m, h, x, w, ps)
        assert rel(host(gX[b]), ox) <= TOL[dt]
        assert rel(host(gH[b]), oh) <= TOL[dt]
