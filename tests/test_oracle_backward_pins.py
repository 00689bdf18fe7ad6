"""Pins for the oracle's gradients of g = H x^{m-1} and f = H x^m.

The paper does not differentiate the product; the reading used throughout is
complex autograd's convention, grad = J^H (cotangent), for these holomorphic
maps.  The oracle's direct-sum gradients are pinned by
* complex autograd (torch, CPU, complex128) through the dense tensor built by
  indexing h (tiny sizes) -- an independent route to J^H v;
* central finite differences of the real loss Re<v, g> + Re(conj(phi) f);
* the dot-product identity <v, J dx> = <J^H v, dx> with J dx evaluated by the
  forward oracle (multilinearity: J dx = (m-1) H dx x^{m-2}).
"""
import numpy as np
import pytest
import torch

from paper_1401_6238_amd import workloads as wl


def torch_dense_grads(m, h, x, v, phi):
    n = len(x)
    ht = torch.tensor(h, dtype=torch.complex128, requires_grad=True)
    xt = torch.tensor(x, dtype=torch.complex128, requires_grad=True)
    idx = torch.tensor(np.indices([n] * m).sum(axis=0))
    T = ht[idx]
    for _ in range(m - 1):
        T = T @ xt
    g = T
    f = torch.dot(xt, g)
    outs, grads = [], []
    if v is not None:
        outs.append(g)
        grads.append(torch.tensor(v, dtype=torch.complex128))
    if phi is not None:
        outs.append(f)
        grads.append(torch.tensor(phi, dtype=torch.complex128))
    gx, gh = torch.autograd.grad(outs, [xt, ht], grads)
    return gx.numpy(), gh.numpy()


@pytest.mark.parametrize("m,n", [(2, 5), (3, 4), (4, 3), (3, 6), (5, 2)])
@pytest.mark.parametrize("which", ["v", "phi", "both"])
def test_backward_vs_complex_autograd(orc, m, n, which):
    g = wl.rng_for(97, m * 100 + n)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0)
    v = wl.cn(g, n, 1.0) if which in ("v", "both") else None
    phi = complex(wl.cn(g, 1, 1.0)[0]) if which in ("phi", "both") else None
    gx, gh = orc.tvp_backward(m, h, x, v, phi)
    tx, th = torch_dense_grads(m, h, x, v, phi)
    assert np.allclose(gx, tx, rtol=1e-12, atol=1e-12)
    assert np.allclose(gh, th, rtol=1e-12, atol=1e-12)


def test_backward_finite_differences(orc):
    m, n = 4, 40
    g = wl.rng_for(98, 0)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])

    def loss(hh, xx):
        y, a = orc.tvp(m, [n] * m, hh, [xx] * m, True, True)
        return float(np.real(np.vdot(v, y)) + np.real(np.conj(phi) * a))

    gx, gh = orc.tvp_backward(m, h, x, v, phi)
    eps = 1e-6
    for l in [0, 7, 39]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            dx = np.zeros(n, np.complex128)
            dx[l] = eps * unit
            fd = (loss(h, x + dx) - loss(h, x - dx)) / (2 * eps)
            assert abs(fd - part(gx[l])) < 1e-7 * max(1.0, abs(gx[l]))
    for s in [0, 50, len(h) - 1]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            dh = np.zeros(len(h), np.complex128)
            dh[s] = eps * unit
            fd = (loss(h + dh, x) - loss(h - dh, x)) / (2 * eps)
            assert abs(fd - part(gh[s])) < 1e-7 * max(1.0, abs(gh[s]))


def test_backward_dot_product_identity(orc):
    m, n = 3, 300
    g = wl.rng_for(99, 0)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    dx = wl.cn(g, n, 1.0)
    dh = wl.cn(g, len(h), 1.0)
    gx, gh = orc.tvp_backward(m, h, x, v, None)
    # J_x dx = (m-1) H dx x^{m-2} (symmetry of the Hankel tensor in modes 2..m)
    jdx, _ = orc.tvp(m, [n] * m, h, [None, dx] + [x] * (m - 2))
    jdh, _ = orc.tvp(m, [n] * m, dh, [None] + [x] * (m - 1))
    lhs_x = np.vdot(v, (m - 1) * jdx)
    rhs_x = np.vdot(gx, dx)
    assert abs(lhs_x - rhs_x) < 1e-11 * abs(lhs_x)
    assert abs(np.vdot(v, jdh) - np.vdot(gh, dh)) < 1e-11 * abs(np.vdot(v, jdh))
