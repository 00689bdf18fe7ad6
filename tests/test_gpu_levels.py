"""GPU parity of level-k block Hankel products (block_hankel_tvp_levels)
against the CPU oracle: levels k = 1..4, equal and distinct vectors, the
scalar product, complex and real dtypes, sizes whose 1D transform is resident
and three-pass; k = 2 also against the native BHHB kernels of
block_hankel_tvp, k = 1 against hankel_mode_products.  Tolerances as in the
other parity tests: relative 2-norm error <= 1e-12 in FP64, <= 1e-4 in FP32."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

DTYPES = [torch.complex64, torch.complex128, torch.float32, torch.float64]


def inputs(seed, m, dims, equal, complex_):
    g = np.random.default_rng(seed)
    k = len(dims)
    d = [sum(dims[t]) - m + 1 for t in range(k)]
    nG = int(np.prod(d))

    def draw(n):
        return (g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)) if complex_ else g.uniform(-1, 1, n)
    G = draw(nG)
    if equal:
        x = draw(int(np.prod([dims[t][0] for t in range(k)])))
        xs = [x] * m
    else:
        xs = [draw(int(np.prod([dims[t][p] for t in range(k)]))) for p in range(m)]
    return G, xs


def run(G, xs, dims, dtype, equal):
    import paper_1401_6238_amd as hk
    Gd = to_dev(G, dtype)
    if equal:
        xd = to_dev(xs[0], dtype)
        vd = [xd] * len(xs)
    else:
        vd = [to_dev(x, dtype) for x in xs]
    y, a = hk.block_hankel_tvp_levels(Gd, vd, dims, True, True)
    torch.cuda.synchronize()
    return host(y), complex(host(a.reshape(1))[0])


CASES = [
    (3, [[5, 5, 5], [3, 3, 3], [2, 2, 2]], True),        # level 3, resident 1D transform
    (3, [[5, 4, 3], [3, 2, 4], [2, 3, 2]], False),
    (2, [[9, 7], [5, 6], [4, 3], [2, 2]], False),       # level 4
    (3, [[20, 14, 17], [12, 9, 10], [6, 4, 5]], False),  # level 3, three-pass 1D transform
    (4, [[12, 12, 12, 12], [10, 10, 10, 10], [5, 5, 5, 5]], True),
    (3, [[64, 64, 64], [40, 40, 40]], True),            # level 2 (BHHB) via the 1D path
    (2, [[1, 1], [1, 1], [1, 1]], False),               # one-entry blocks
]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,dims,equal", CASES)
def test_levels_vs_oracle(dtype, m, dims, equal):
    print_case(test="levels", dtype=dtype, m=m, dims=dims, equal=equal)
    G, xs = inputs(len(dims) * 100 + m + sum(map(sum, dims)), m, dims, equal, dtype.is_complex)
    y, a = run(G, xs, dims, dtype, equal)
    yo, ao = oracle.block_levels_tvp(m, dims, seen(G, dtype), [seen(x, dtype) for x in xs], True, True)
    assert rel(y, yo) <= TOL[dtype]
    check_alpha(a, ao, dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_level2_matches_native_bhhb(dtype):
    import paper_1401_6238_amd as hk
    m, dims = 3, [[40, 33, 25], [30, 21, 17]]
    print_case(test="level2_vs_bhhb", dtype=dtype)
    G, xs = inputs(7, m, dims, False, True)
    y, a = run(G, xs, dims, dtype, False)
    yb, ab = hk.block_hankel_tvp(to_dev(G, dtype), [to_dev(x, dtype) for x in xs], dims[0], dims[1], True, True)
    torch.cuda.synchronize()
    # both paths against the BHHB oracle (the level-2 generating tensor is the BHHB generating matrix)
    yo, ao = oracle.block_tvp(m, dims[0], dims[1], seen(G, dtype), [seen(x, dtype) for x in xs], True, True)
    for yy, aa in ((y, a), (host(yb), complex(host(ab.reshape(1))[0]))):
        assert rel(yy, yo) <= TOL[dtype]
        check_alpha(aa, ao, dtype)


def test_level1_matches_mode_products():
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    m, dims = 4, [[300, 250, 200, 280]]
    G, xs = inputs(8, m, dims, False, True)
    y, a = run(G, xs, dims, dtype, False)
    y1, a1 = hk.hankel_mode_products(to_dev(G, dtype), [to_dev(x, dtype) for x in xs], dims[0], True, True)
    torch.cuda.synchronize()
    # both paths against the 1D oracle (a level-1 tensor is a Hankel tensor)
    yo, ao = oracle.tvp(m, dims[0], seen(G, dtype), [seen(x, dtype) for x in xs], True, True)
    for yy, aa in ((y, a), (host(y1), complex(host(a1.reshape(1))[0]))):
        assert rel(yy, yo) <= TOL[dtype]
        check_alpha(aa, ao, dtype)
