"""GPU parity of the spectral form (hankel_spectrum, hankel_mode_products_spectral)
against the CPU oracle.  Spectra are compared with the oracle's DFT sums of
Section 3's h^ = ifft(pad_N h) and x^ = fft(pad_N x), through the documented
row order (element r R + c holds bin r + C c); products made from spectra are
compared with the direct products.  Shapes with R = C, R = 2 C and R = 4 C, spectra of
all operands, of some (mixed with plain vectors) or of h only (the warm single
product), equal vectors merged into powers, and the scalar product.
Tolerances as in the other parity tests: relative 2-norm error <= 1e-12 in
FP64, <= 1e-4 in FP32 (scalar: 10x)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

CDTYPES = [torch.complex64, torch.complex128]
DTYPES = CDTYPES + [torch.float32, torch.float64]


def draw(g, n, scale=1.0, real=False):
    if real:
        return g.uniform(-1, 1, n) * scale
    return (g.standard_normal(n) + 1j * g.standard_normal(n)) * scale


def bins_of_layout(N, R):
    """Bin held by each spectrum element: element r R + c holds bin r + C c."""
    C = N // R
    e = np.arange(N)
    return (e // R) + C * (e % R)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n", [(3, 3000), (4, 8192), (4, 16384)])
def test_spectra_match_dft(dtype, m, n):
    """Real dtypes: the spectra of real data, complex values of the same precision."""
    import paper_1401_6238_amd as hk
    print_case(test="spectra", dtype=dtype, m=m, n=n)
    g = np.random.default_rng(100 + m)
    dims = [n] * m
    dh = m * (n - 1) + 1
    real = not dtype.is_complex
    h, x = draw(g, dh, real=real), draw(g, n, 1.0 / n, real=real)
    N, R = hk.hankel_spectrum_layout(dtype, m, dims)
    assert N >= dh and N & (N - 1) == 0 and N // 2 < dh
    sh = hk.hankel_spectrum(to_dev(h, dtype), m, dims, -1)
    sx = hk.hankel_spectrum(to_dev(x, dtype), m, dims, 2)
    torch.cuda.synchronize()
    assert sh.is_complex() and sh.numel() == N
    # a sample of elements that covers whole rows at both ends and scattered ones
    sel = np.unique(np.concatenate([np.arange(2 * R), np.arange(N - 2 * R, N),
                                    np.random.default_rng(7).integers(0, N, 2048)]))
    b = bins_of_layout(N, R)[sel]
    ref_h = oracle.spectrum(seen(h, dtype), N, b, inverse=True)
    ref_x = oracle.spectrum(seen(x, dtype), N, b)
    assert rel(host(sh)[sel], ref_h) <= TOL[dtype]
    assert rel(host(sx)[sel], ref_x) <= TOL[dtype]


@pytest.mark.parametrize("dtype", CDTYPES)
@pytest.mark.parametrize("kind", ["all_spectra", "mixed", "h_only", "equal_powers"])
def test_products_from_spectra(dtype, kind):
    import paper_1401_6238_amd as hk
    print_case(test="spectral_products", dtype=dtype, kind=kind)
    g = np.random.default_rng({"all_spectra": 1, "mixed": 2, "h_only": 3, "equal_powers": 4}[kind])
    if kind == "equal_powers":
        m, dims = 4, [6000] * 4
    else:
        m, dims = 3, [2500, 3100, 1800]
    dh = sum(dims) - m + 1
    h = draw(g, dh)
    if kind == "equal_powers":
        x = draw(g, dims[0], 1.0 / dims[0])
        xs = [x] * m
    else:
        xs = [draw(g, n, 1.0 / n) for n in dims]
    hd = to_dev(h, dtype)
    xd = [to_dev(v, dtype) for v in xs]
    if kind == "equal_powers":
        xd = [xd[0]] * m
    hs = hk.hankel_spectrum(hd, m, dims, -1)
    if kind == "all_spectra":
        specs = [hk.hankel_spectrum(xd[p], m, dims, p) for p in range(m)]
        vectors = None
    elif kind == "mixed":
        specs = [None, hk.hankel_spectrum(xd[1], m, dims, 1), None]
        vectors = xd
    elif kind == "h_only":
        specs, vectors = None, xd
    else:
        s = hk.hankel_spectrum(xd[0], m, dims, 0)
        specs, vectors = [s] * m, None
    y, a = hk.hankel_mode_products_spectral(hs, m, dims, vectors, specs, True, True)
    torch.cuda.synchronize()
    yo, ao = oracle.tvp(m, dims, seen(h, dtype), [seen(v, dtype) for v in xs], True, True)
    assert rel(host(y), yo) <= TOL[dtype]
    a = complex(host(a.reshape(1))[0])
    check_alpha(a, ao, dtype)


@pytest.mark.parametrize("dtype", CDTYPES)
def test_warm_products(dtype):
    """h^ made once serves several new vectors (N = 2^16, rows of 2^9): sampled
    outputs and the scalar of each product against the oracle."""
    import paper_1401_6238_amd as hk
    print_case(test="warm_products", dtype=dtype)
    g = np.random.default_rng(11)
    m, n = 4, 1 << 14
    dims = [n] * m
    h = draw(g, m * (n - 1) + 1)
    hs = hk.hankel_spectrum(to_dev(h, dtype), m, dims, -1)
    idx = np.unique(np.concatenate([np.arange(16), np.arange(n - 16, n), g.integers(0, n, 64)]))
    for k in range(2):
        x = draw(g, n, 1.0 / n)
        xd = to_dev(x, dtype)
        y, a = hk.hankel_mode_products_spectral(hs, m, dims, [xd] * m, None, True, True)
        torch.cuda.synchronize()
        xo = seen(x, dtype)
        yo, ao = oracle.tvp_sampled(m, dims, seen(h, dtype), [xo] * m, idx, want_alpha=True)
        assert rel(host(y)[idx], yo) <= TOL[dtype]
        check_alpha(complex(a), ao, dtype)


@pytest.mark.parametrize("dtype", CDTYPES)
@pytest.mark.parametrize("m,n", [(3, 8000), (4, 1 << 14)])
def test_spectral_strided_batch(dtype, m, n):
    """One stored h^ shared by a strided batch of 5 vectors: every instance's
    scalar and sampled outputs against the oracle."""
    import paper_1401_6238_amd as hk
    print_case(test="spectral_strided_batch", dtype=dtype, m=m, n=n)
    g = np.random.default_rng(21 + m)
    B = 5
    h = draw(g, m * (n - 1) + 1)
    X = np.stack([draw(g, n, 1.0 / n) for _ in range(B)])
    hs = hk.hankel_spectrum(to_dev(h, dtype), m, [n] * m, -1)
    Xd = to_dev(X.reshape(-1), dtype).reshape(B, n)
    Y, A = hk.hankel_tvp_spectral_strided_batched(hs, Xd, m, True, True)
    torch.cuda.synchronize()
    Y, A = host(Y), host(A)
    idx = np.unique(np.concatenate([np.arange(8), np.arange(n - 8, n), g.integers(0, n, 32)]))
    ho = seen(h, dtype)
    for b in range(B):
        xo = seen(X[b], dtype)
        yo, ao = oracle.tvp_sampled(m, [n] * m, ho, [xo] * m, idx, want_alpha=True)
        assert rel(Y[b][idx], yo) <= TOL[dtype], b
        check_alpha(A[b], ao, dtype, b)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_real_products_from_spectra(dtype):
    """Real h and vectors: products from h^ and one stored vector spectrum are
    real, against the oracle; the warm strided batch on real data too."""
    import paper_1401_6238_amd as hk
    print_case(test="real_spectral_products", dtype=dtype)
    g = np.random.default_rng(31)
    m, dims = 3, [2500, 3100, 1800]
    h = draw(g, sum(dims) - m + 1, real=True)
    xs = [draw(g, n, real=True) for n in dims]
    xd = [to_dev(v, dtype) for v in xs]
    hs = hk.hankel_spectrum(to_dev(h, dtype), m, dims, -1)
    specs = [None, hk.hankel_spectrum(xd[1], m, dims, 1), None]
    y, a = hk.hankel_mode_products_spectral(hs, m, dims, xd, specs, True, True)
    torch.cuda.synchronize()
    assert y.dtype == dtype and not torch.is_complex(a)
    yo, ao = oracle.tvp(m, dims, seen(h, dtype), [seen(v, dtype) for v in xs], True, True)
    assert rel(host(y), yo) <= TOL[dtype]
    check_alpha(float(a), ao, dtype)
    # warm strided batch, m = 4, n = 2^13
    m, n, B = 4, 1 << 13, 3
    h = draw(g, m * (n - 1) + 1, real=True)
    X = np.stack([draw(g, n, real=True) for _ in range(B)])
    hs = hk.hankel_spectrum(to_dev(h, dtype), m, [n] * m, -1)
    Y, A = hk.hankel_tvp_spectral_strided_batched(hs, to_dev(X.reshape(-1), dtype).reshape(B, n), m, True, True)
    torch.cuda.synchronize()
    assert Y.dtype == dtype
    idx = np.unique(np.concatenate([np.arange(8), np.arange(n - 8, n), g.integers(0, n, 32)]))
    for b in range(B):
        yo, ao = oracle.tvp_sampled(m, [n] * m, seen(h, dtype), [seen(X[b], dtype)] * m, idx, want_alpha=True)
        assert rel(host(Y[b])[idx], yo) <= TOL[dtype], b
        check_alpha(float(A[b]), ao, dtype, b)


@pytest.mark.parametrize("want", ["y", "alpha"])
def test_spectral_single_output(want):
    """Only y or only alpha requested from stored spectra."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    print_case(test="spectral_single_output", want=want)
    g = np.random.default_rng(41)
    m, dims = 3, [3000, 2600, 2200]
    h = draw(g, sum(dims) - m + 1)
    xs = [draw(g, n, 1.0 / n) for n in dims]
    xd = [to_dev(v, dtype) for v in xs]
    hs = hk.hankel_spectrum(to_dev(h, dtype), m, dims, -1)
    specs = [hk.hankel_spectrum(xd[p], m, dims, p) for p in range(m)]
    y, a = hk.hankel_mode_products_spectral(hs, m, dims, None, specs, want == "y", want == "alpha")
    torch.cuda.synchronize()
    yo, ao = oracle.tvp(m, dims, seen(h, dtype), [seen(v, dtype) for v in xs], True, True)
    if want == "y":
        assert a is None and rel(host(y), yo) <= TOL[dtype]
    else:
        assert y is None
        check_alpha(complex(a), ao, dtype)


@pytest.mark.parametrize("dtype", CDTYPES)
@pytest.mark.parametrize("m,n", [(3, 4000), (4, 1 << 14)])
def test_backward_with_stored_x_spectrum(dtype, m, n):
    """The adjoint from a stored x^ (the forward's spectrum kept): grad_x and
    grad_h against the oracle, with both cotangents and with grad_h alone."""
    import paper_1401_6238_amd as hk
    print_case(test="backward_spectral", dtype=dtype, m=m, n=n)
    g = np.random.default_rng(51 + m)
    h = draw(g, m * (n - 1) + 1)
    x = draw(g, n, 1.0 / n)
    v = draw(g, n)
    phi = complex(draw(g, 1)[0])
    hd, xd, vd = to_dev(h, dtype), to_dev(x, dtype), to_dev(v, dtype)
    phd = to_dev(np.array([phi]), dtype)
    xs = hk.hankel_spectrum(xd, m, [n] * m, 1)
    gx, gh = hk.hankel_tvp_backward_spectral(hd, xs, m, n, vd, phd, True, True)
    _, gh_only = hk.hankel_tvp_backward_spectral(hd, xs, m, n, None, phd, False, True)
    torch.cuda.synchronize()
    gxo, gho = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), seen(v, dtype), complex(seen(np.array([phi]), dtype)[0]))
    assert rel(host(gx), gxo) <= TOL[dtype]
    assert rel(host(gh), gho) <= TOL[dtype]
    _, gho2 = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), None, complex(seen(np.array([phi]), dtype)[0]),
                                  want_grad_x=False)
    assert rel(host(gh_only), gho2) <= TOL[dtype]
