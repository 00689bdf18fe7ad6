"""Forward products that keep x^ for the adjoint (hankel_tvp_save_spectrum),
the strided batch of the adjoint from stored spectra, and the autograd path
that joins them, against the CPU oracle: y and alpha against the direct
products, the saved spectra against the oracle's DFT sums of Section 3's
x^ = fft(pad_N x) through the documented row order, gradients against the
oracle's direct-sum gradients.  Tolerances: relative 2-norm error <= 1e-12
in FP64, <= 1e-4 in FP32 (alpha: |d alpha| / |alpha| at the same bound)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

CDTYPES = [torch.complex64, torch.complex128]


def draw(g, n, scale=1.0):
    return (g.standard_normal(n) + 1j * g.standard_normal(n)) * scale


def bins_of_layout(N, R):
    """Bin held by each spectrum element: element r R + c holds bin r + C c."""
    C = N // R
    e = np.arange(N)
    return (e // R) + C * (e % R)


def instance(seed, m, n):
    g = np.random.default_rng(seed)
    return draw(g, m * (n - 1) + 1), draw(g, n, 1.0 / n), draw(g, n), complex(draw(g, 1)[0])


@pytest.mark.parametrize("dtype", CDTYPES)
@pytest.mark.parametrize("m,n,B", [(3, 3000, 1), (4, 2500, 3), (4, 1 << 14, 2)])
def test_save_spectrum_forward(dtype, m, n, B):
    import paper_1401_6238_amd as hk
    print_case(test="save_spectrum", dtype=dtype, m=m, n=n, B=B)
    data = [instance(900 + 7 * b + m, m, n) for b in range(B)]
    H = torch.stack([to_dev(d[0], dtype) for d in data])
    X = torch.stack([to_dev(d[1], dtype) for d in data])
    if B == 1:
        y, a, spec = hk.hankel_tvp_save_spectrum(H[0], X[0], m, True, True)
        y, a, spec = y.reshape(1, -1), a.reshape(1), spec.reshape(1, -1)
    else:
        y, a, spec = hk.hankel_tvp_save_spectrum(H, X, m, True, True)
    torch.cuda.synchronize()
    N, R = hk.hankel_spectrum_layout(dtype, m, [n] * m)
    assert spec.shape == (B, N)
    sel = np.unique(np.concatenate([np.arange(2 * R), np.arange(N - 2 * R, N),
                                    np.random.default_rng(8).integers(0, N, 2048)]))
    bins = bins_of_layout(N, R)[sel]
    for b, (h, x, _, _) in enumerate(data):
        hs, xs = seen(h, dtype), seen(x, dtype)
        yo, ao = oracle.tvp(m, [n] * m, hs, [xs] * m, True, True)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        check_alpha(complex(host(a[b:b + 1])[0]), ao, dtype, f"instance {b}")
        assert rel(host(spec[b])[sel], oracle.spectrum(xs, N, bins)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", CDTYPES)
@pytest.mark.parametrize("cot", ["both", "v", "phi"])
def test_backward_spectral_strided_batched(dtype, cot):
    """The batched adjoint from the spectra the forward saved, every instance
    against the oracle's gradients."""
    import paper_1401_6238_amd as hk
    m, n, B = 4, 2500, 3
    print_case(test="backward_spectral_batched", dtype=dtype, cot=cot)
    data = [instance(950 + b, m, n) for b in range(B)]
    H = torch.stack([to_dev(d[0], dtype) for d in data])
    X = torch.stack([to_dev(d[1], dtype) for d in data])
    V = torch.stack([to_dev(d[2], dtype) for d in data]) if cot != "phi" else None
    P = to_dev(np.array([d[3] for d in data]), dtype) if cot != "v" else None
    _, _, spec = hk.hankel_tvp_save_spectrum(H, X, m, False, True)
    gx, gh = hk.hankel_tvp_backward_spectral_strided_batched(H, spec, m, n, V, P)
    torch.cuda.synchronize()
    for b, (h, x, v, phi) in enumerate(data):
        vs = seen(v, dtype) if cot != "phi" else None
        ps = complex(seen(np.array([phi]), dtype)[0]) if cot != "v" else None
        ox, oh = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), vs, ps)
        assert rel(host(gx[b]), ox) <= TOL[dtype]
        assert rel(host(gh[b]), oh) <= TOL[dtype]


@pytest.mark.parametrize("batched", [False, True])
def test_autograd_reuses_saved_spectrum(batched):
    """Autograd on a shape with the spectral layout (d_H > 4096): the forward
    keeps x^ and the backward reads it; gradients of h and x, and of x alone,
    against the oracle."""
    import paper_1401_6238_amd as hk
    m, n = 4, 2000
    dt = torch.complex128
    B = 2 if batched else 1
    data = [instance(970 + b, m, n) for b in range(B)]
    H = torch.stack([to_dev(d[0], dt) for d in data]).requires_grad_(True)
    X = torch.stack([to_dev(d[1], dt) for d in data]).requires_grad_(True)
    V = torch.stack([to_dev(d[2], dt) for d in data])
    P = to_dev(np.array([d[3] for d in data]), dt)
    hh, xx, vv, pp = (H, X, V, P) if batched else (H[0], X[0], V[0], P[0])
    g, f = hk.hankel_tvp_autograd(hh, xx, m)
    gH, gX = torch.autograd.grad([g, f], [H, X], [vv, pp])
    for b, (h, x, v, phi) in enumerate(data):
        ox, oh = oracle.tvp_backward(m, h, x, v, phi)
        assert rel(host(gX[b]), ox) <= TOL[dt]
        assert rel(host(gH[b]), oh) <= TOL[dt]
    # x alone requires grad: the forward still keeps x^ (grad_x needs h^ only,
    # grad_h is not requested)
    xt = to_dev(data[0][1], dt).requires_grad_(True)
    g, f = hk.hankel_tvp_autograd(to_dev(data[0][0], dt), xt, m)
    (gx,) = torch.autograd.grad([g, f], [xt], [to_dev(data[0][2], dt), torch.tensor(data[0][3], dtype=dt,
                                                                                    device=xt.device)])
    ox, _ = oracle.tvp_backward(m, *data[0])
    assert rel(host(gx), ox) <= TOL[dt]
