"""Pins for the oracle's gradients of the products with distinct vectors,
1D (y = H x_2 ... x_m, alpha = H x_1 ... x_m) and BHHB (the same with the
2-level block tensor of Section 2.2 and vec(X_p), vec(Y)).

The paper does not differentiate; the reading is complex autograd's
convention, grad = J^H (cotangent).  Each oracle gradient is pinned by
* complex autograd (torch, CPU, complex128) through the dense tensor built by
  indexing h or H (tiny sizes, non-square dims with n_p != N_p) -- a route
  that shares nothing with the oracle's convolution/correlation sums;
* the equal-vector adjoint: with x_1 = ... = x_m the gradients of the
  distinct vectors add up to the equal-vector gradient (chain rule);
* the dot-product identity <v, J_p dx> = <grad_p, dx>, J_p dx evaluated by
  the forward oracle (the product is linear in x_p).
"""
import numpy as np
import pytest
import torch

from paper_1401_6238_amd import workloads as wl


def dense_1d(m, dims, h):
    idx = torch.tensor(np.indices(dims).sum(axis=0))
    return h[idx]


def dense_block(m, dims, bdims, H):
    """T[a_1, ..., a_m] = H[i_1 + ... + i_m, j_1 + ... + j_m] with
    a_p = i_p + n_p j_p (column-major vec of the n_p x N_p block index)."""
    shape = []
    for p in range(m):
        shape += [dims[p], bdims[p]]
    ind = np.indices(shape)
    rows = sum(ind[2 * p] for p in range(m))
    cols = sum(ind[2 * p + 1] for p in range(m))
    T = H[torch.tensor(rows), torch.tensor(cols)]
    # reorder each (i_p, j_p) pair to a_p = i_p + n_p j_p: transpose to (j_p, i_p) then flatten
    perm = []
    for p in range(m):
        perm += [2 * p + 1, 2 * p]
    T = T.permute(perm)
    return T.reshape([dims[p] * bdims[p] for p in range(m)])


def torch_grads(T_of, params, xs, v, phi):
    xt = [torch.tensor(x, dtype=torch.complex128, requires_grad=True) for x in xs]
    T = T_of(params)
    y = T
    for q in range(len(xs) - 1, 0, -1):
        y = y @ xt[q]
    outs, cots = [], []
    if v is not None:
        outs.append(y)
        cots.append(torch.tensor(v, dtype=torch.complex128))
    if phi is not None:
        outs.append(torch.dot(xt[0], y))
        cots.append(torch.tensor(phi, dtype=torch.complex128))
    grads = torch.autograd.grad(outs, xt + [params], cots, allow_unused=True)
    return [None if g is None else g.numpy() for g in grads]


@pytest.mark.parametrize("dims", [(4, 3), (3, 4, 2), (2, 3, 2, 3), (3, 2, 2, 1, 2)])
@pytest.mark.parametrize("which", ["v", "phi", "both"])
def test_mode_backward_vs_complex_autograd(orc, dims, which):
    m = len(dims)
    g = wl.rng_for(99, sum(dims) * 10 + m)
    dh = sum(dims) - m + 1
    h = wl.cn(g, dh, 1.0)
    xs = [wl.cn(g, n, 1.0) for n in dims]
    v = wl.cn(g, dims[0], 1.0) if which != "phi" else None
    phi = complex(wl.cn(g, 1, 1.0)[0]) if which != "v" else None
    gv, gh = orc.mode_backward(m, dims, h, xs, v, phi)
    ht = torch.tensor(h, dtype=torch.complex128, requires_grad=True)
    tg = torch_grads(lambda hh: dense_1d(m, dims, hh), ht, xs, v, phi)
    for p in range(m):
        ref = tg[p] if tg[p] is not None else np.zeros(dims[p], np.complex128)
        assert np.allclose(gv[p], ref, rtol=1e-12, atol=1e-12), p
    assert np.allclose(gh, tg[m], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,bdims", [((2, 3), (3, 2)), ((2, 3, 2), (3, 2, 2)), ((1, 2, 2), (2, 1, 3))])
@pytest.mark.parametrize("which", ["v", "phi", "both"])
def test_block_backward_vs_complex_autograd(orc, dims, bdims, which):
    m = len(dims)
    g = wl.rng_for(100, sum(dims) * 10 + sum(bdims))
    hr, hc = sum(dims) - m + 1, sum(bdims) - m + 1
    H = wl.cn(g, hr * hc, 1.0)  # column-major hr x hc
    xs = [wl.cn(g, dims[p] * bdims[p], 1.0) for p in range(m)]
    v = wl.cn(g, dims[0] * bdims[0], 1.0) if which != "phi" else None
    phi = complex(wl.cn(g, 1, 1.0)[0]) if which != "v" else None
    gv, gH = orc.block_backward(m, dims, bdims, H, xs, v, phi)
    Ht = torch.tensor(H.reshape(hc, hr).T.copy(), dtype=torch.complex128, requires_grad=True)  # Ht[r, c]
    tg = torch_grads(lambda HH: dense_block(m, dims, bdims, HH), Ht, xs, v, phi)
    for p in range(m):
        ref = tg[p] if tg[p] is not None else np.zeros(dims[p] * bdims[p], np.complex128)
        assert np.allclose(gv[p], ref, rtol=1e-12, atol=1e-12), p
    assert np.allclose(gH, tg[m].T.reshape(-1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m,n", [(2, 40), (3, 30), (4, 25)])
def test_mode_backward_equal_vectors_add_up(orc, m, n):
    """x_1 = ... = x_m: the chain rule sums the distinct-vector gradients into
    the equal-vector gradient of the oracle's tvp_backward."""
    g = wl.rng_for(101, m)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    gv, gh = orc.mode_backward(m, [n] * m, h, [x] * m, v, phi)
    ex, eh = orc.tvp_backward(m, h, x, v, phi)
    assert np.allclose(sum(gv), ex, rtol=1e-12, atol=1e-12 * np.abs(ex).max())
    assert np.allclose(gh, eh, rtol=1e-12, atol=1e-12 * np.abs(eh).max())


def test_block_backward_equal_vectors_add_up(orc):
    """BHHB with equal vectors against the 1D equal-vector adjoint of a level-2
    tensor whose blocks are 1 x N (n_p = 1 reduces BHHB to a 1D Hankel tensor
    along the block index)."""
    m, N = 3, 9
    g = wl.rng_for(102, 0)
    h = wl.cn(g, m * (N - 1) + 1, 1.0)
    x = wl.cn(g, N, 1.0 / N)
    v = wl.cn(g, N, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    gv, gH = orc.block_backward(m, [1] * m, [N] * m, h, [x] * m, v, phi)
    ex, eh = orc.tvp_backward(m, h, x, v, phi)
    assert np.allclose(sum(gv), ex, rtol=1e-12, atol=1e-13)
    assert np.allclose(gH, eh, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("p", [0, 1, 2])
def test_mode_backward_dot_product_identity(orc, p):
    """<v, J_p dx> + conj(phi) (d alpha) = <grad_p, dx>: J_p dx is the forward
    oracle with x_p replaced by dx (the products are linear in x_p)."""
    dims = [30, 22, 17]
    m = 3
    g = wl.rng_for(103, p)
    h = wl.cn(g, sum(dims) - m + 1, 1.0)
    xs = [wl.cn(g, n, 1.0) for n in dims]
    v = wl.cn(g, dims[0], 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    dx = wl.cn(g, dims[p], 1.0)
    gv, _ = orc.mode_backward(m, dims, h, xs, v, phi)
    xd = list(xs)
    xd[p] = dx
    y, a = orc.tvp(m, dims, h, xd, True, True)
    lhs = (np.vdot(v, y) if p > 0 else 0.0) + np.conj(phi) * a
    rhs = np.vdot(gv[p], dx)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
