"""GPU parity of the plain path (resident and 3-pass) against the CPU oracle.

Sizes are chosen so that the oracle finishes in seconds while the transforms
still span several tiles, passes and ragged tails.  Tolerances: relative
2-norm error <= 1e-12 in FP64 and <= 1e-4 in FP32 (complex or real).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, oracle_problem, print_case, rel, seen, to_dev  # noqa: E402

DTYPES = [torch.complex128, torch.complex64]


def run_problem(prob, dtype):
    import paper_1401_6238_amd as hk
    h = to_dev(prob.h, dtype)
    vecs = [to_dev(v, dtype) if v is not None else None for v in prob.vectors]
    if prob.is_block:
        y, a = hk.block_hankel_tvp(h, vecs, prob.dims, prob.block_dims, prob.want_y, prob.want_alpha)
    elif prob.equal and prob.vectors[1] is not None:
        y, a = hk.hankel_tvp(h, vecs[1], prob.m, prob.want_y, prob.want_alpha)
    else:
        y, a = hk.hankel_mode_products(h, vecs, prob.dims, prob.want_y, prob.want_alpha)
    torch.cuda.synchronize()
    return host(y), (None if a is None else complex(host(a.reshape(1))[0]))


def check(prob, dtype, tol=None):
    tol = TOL[dtype] if tol is None else tol
    y, a = run_problem(prob, dtype)
    yo, ao = oracle_problem(prob, dtype)
    if prob.want_y:
        e = rel(y, yo)
        assert e <= tol, f"y rel err {e:.3e} > {tol}"
    if prob.want_alpha:
        check_alpha(a, ao, dtype, tol=tol)


def test_small_real_f64():
    """m=3, n=64, real FP64 inputs (the small published-shape case)."""
    prob = wl.small_real()
    print_case(test="small_real", dtype="f64")
    check(prob, torch.float64)


@pytest.mark.parametrize("dtype", DTYPES + [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n", [(2, 1), (2, 2), (3, 1), (2, 5), (3, 7), (4, 16), (3, 64), (5, 100), (2, 2048),
                                 (3, 1000), (4, 1365), (8, 10)])
def test_resident_equal(dtype, m, n):
    print_case(test="resident_equal", dtype=dtype, m=m, n=n)
    prob = wl.random_problem(1000 + 7 * m + n, m, [n] * m, True, complex_=dtype.is_complex, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,dims", [(2, [9, 4]), (3, [5, 1, 9]), (4, [30, 2, 17, 8]), (5, [3, 40, 1, 7, 2]),
                                    (3, [1000, 700, 1200]), (2, [1, 3000])])
@pytest.mark.parametrize("kind", ["y", "alpha", "both"])
def test_resident_distinct(dtype, m, dims, kind):
    print_case(test="resident_distinct", dtype=dtype, m=m, dims=dims, kind=kind)
    prob = wl.random_problem(2000 + sum(dims), m, dims, False, want_y=kind != "alpha",
                             want_alpha=kind != "y")
    check(prob, dtype)


@pytest.mark.parametrize("dtype", DTYPES + [torch.float64])
@pytest.mark.parametrize("m,n", [(3, 2049), (4, 3000), (3, 4096), (2, 20000), (5, 3333)])
def test_multipass_equal(dtype, m, n):
    print_case(test="multipass_equal", dtype=dtype, m=m, n=n)
    prob = wl.random_problem(3000 + m * n, m, [n] * m, True, complex_=dtype.is_complex, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,dims", [(3, [5000, 3, 4000]), (4, [2500, 1700, 1, 2600]), (2, [7000, 9000]),
                                    (3, [1, 6000, 5000])])
def test_multipass_distinct(dtype, m, dims):
    print_case(test="multipass_distinct", dtype=dtype, m=m, dims=dims)
    prob = wl.random_problem(4000 + sum(dims), m, dims, False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("m,n", [(3, 64), (4, 24), (3, 2000), (2, 6000)])
def test_integer_exact_c128(m, n):
    """Integer inputs: rounded FP64 GPU results equal the complex-int64 oracle bit for bit."""
    print_case(test="integer_exact", m=m, n=n)
    prob = wl.random_problem(5000 + n, m, [n] * m, True, want_alpha=True, integer=3)
    y, a = run_problem(prob, torch.complex128)
    yi, ai = oracle.tvp_i64(m, prob.dims, prob.h, prob.vectors, True, True)
    assert np.max(np.abs(yi)) < 2 ** 40
    assert np.array_equal(np.round(y.real).astype(np.int64), yi[:, 0])
    assert np.array_equal(np.round(y.imag).astype(np.int64), yi[:, 1])
    assert (round(a.real), round(a.imag)) == (ai[0], ai[1])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,dims,bdims", [(2, [2, 3], [3, 2]), (3, [3, 3, 3], [2, 2, 2]), (3, [20, 20, 20], [13, 13, 13]),
                                          (3, [7, 2, 5], [3, 9, 4]), (2, [1, 40], [30, 1]), (4, [5, 6, 7, 8], [4, 3, 2, 1])])
def test_block(dtype, m, dims, bdims):
    print_case(test="block", dtype=dtype, m=m, dims=dims, bdims=bdims)
    prob = wl.random_problem(6000 + sum(dims) + 3 * sum(bdims), m, dims, False, want_alpha=True, block_dims=bdims)
    check(prob, dtype)


def test_block_equal_vectors():
    print_case(test="block_equal")
    prob = wl.random_problem(6100, 3, [30, 30, 30], True, want_alpha=True, block_dims=[25, 25, 25])
    check(prob, torch.complex128)
