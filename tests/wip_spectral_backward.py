"""Adjoint from a stored x spectrum, against the oracle (kept out of the
collected tests until it has run on the GPU)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402

CDTYPES = [torch.complex64, torch.complex128]


def draw(g, n, scale=1.0):
    return (g.standard_normal(n) + 1j * g.standard_normal(n)) * scale


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
