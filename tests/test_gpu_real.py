"""GPU parity of the real-input forward path against the CPU oracle.  Real
forward products transform each real vector of padded length N as N/2
complex pairs (length-N/2 complex FFT, then the split into the real
transform's half spectrum by conjugate symmetry), multiply on bins 0..N/2 and
return the real result packed in pairs: in one workgroup up to N = 8192
(float) / 4096 (double), in three passes beyond (the row pass on mirrored row
pairs).  These cases cover the degenerate lengths (N = 2, 4),
odd and even d_H and output lengths, every row length, equal and distinct
vectors, the scalar product (a half-spectrum sum), strided batches and
grouped plans (also against the complex path of a power-of-two-only plan).
Tolerances as in the other parity tests: relative 2-norm error <= 1e-12 in
FP64, <= 1e-4 in FP32."""
import numpy as np
import pytest
import torch

from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, oracle_problem, print_case, rel, to_dev  # noqa: E402
from test_gpu_batched import check_plan_outputs, plan_inputs  # noqa: E402
from test_gpu_parity import check  # noqa: E402

REAL = [torch.float32, torch.float64]


EQUAL_SHAPES = [(2, 1), (2, 2), (3, 2), (2, 3), (3, 3), (4, 4), (3, 7), (2, 64), (3, 64), (5, 33),
                (3, 100), (4, 300), (3, 683), (2, 2048), (3, 1366), (4, 1365), (5, 1024), (3, 2731), (8, 500)]
# resident real rows hold N <= 8192 (float) and N <= 4096 (double); the double
# shapes beyond that run three passes, which test_multipass_equal covers
EQUAL_CASES = [(dt, m, n) for dt in REAL for (m, n) in EQUAL_SHAPES
               if not (dt == torch.float64 and m * (n - 1) + 1 > 4096)]


@pytest.mark.parametrize("dtype,m,n", EQUAL_CASES)
def test_equal(dtype, m, n):
    print_case(test="real_equal", dtype=dtype, m=m, n=n)
    prob = wl.random_problem(9500 + 7 * m + n, m, [n] * m, True, complex_=False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", REAL)
@pytest.mark.parametrize("dims", [[5, 3, 2], [64, 40, 20], [700, 300, 900], [1000, 1500, 1200, 800], [2, 1]])
def test_distinct(dtype, dims):
    m = len(dims)
    print_case(test="real_distinct", dtype=dtype, dims=dims)
    prob = wl.random_problem(9600 + sum(dims), m, dims, False, complex_=False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", REAL)
@pytest.mark.parametrize("m,n,B", [(3, 64, 9), (3, 1000, 5), (4, 1365, 3)])
def test_strided_batched(dtype, m, n, B):
    import paper_1401_6238_amd as hk
    print_case(test="real_strided", dtype=dtype, m=m, n=n, B=B)
    probs = [wl.random_problem(9700 + b, m, [n] * m, True, complex_=False, want_alpha=True) for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        yo, ao = oracle_problem(p, dtype)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        check_alpha(complex(host(a[b:b + 1])[0]), ao, dtype)


@pytest.mark.parametrize("dtype", REAL)
@pytest.mark.parametrize("m,n", [(3, 2800), (3, 4000), (4, 5000), (5, 3000), (2, 40000), (3, 30000), (8, 2000)])
def test_multipass_equal(dtype, m, n):
    print_case(test="real_multipass_equal", dtype=dtype, m=m, n=n)
    prob = wl.random_problem(9900 + 7 * m + n, m, [n] * m, True, complex_=False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", REAL)
@pytest.mark.parametrize("dims", [[5000, 3000, 4001], [20000, 9999], [3001, 2000, 2500, 1800]])
def test_multipass_distinct(dtype, dims):
    m = len(dims)
    print_case(test="real_multipass_distinct", dtype=dtype, dims=dims)
    prob = wl.random_problem(9950 + sum(dims), m, dims, False, complex_=False, want_alpha=True)
    check(prob, dtype)


@pytest.mark.parametrize("dtype", REAL)
def test_multipass_strided(dtype):
    import paper_1401_6238_amd as hk
    m, n, B = 3, 5000, 3
    print_case(test="real_multipass_strided", dtype=dtype)
    probs = [wl.random_problem(9990 + b, m, [n] * m, True, complex_=False, want_alpha=True) for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        yo, ao = oracle_problem(p, dtype)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        check_alpha(complex(host(a[b:b + 1])[0]), ao, dtype)


@pytest.mark.parametrize("dtype", REAL)
def test_plan(dtype):
    """A grouped plan of real problems of many sizes (real rows, and the
    complex path beyond one workgroup) against the oracle, and the same plan
    restricted to powers of two (complex path) against the oracle too."""
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    print_case(test="real_plan", dtype=dtype)
    g = np.random.Generator(np.random.PCG64(97))
    probs = []
    for i in range(40):
        m = int(g.integers(2, 6))
        n = int(np.exp(g.uniform(np.log(2), np.log(12000))))
        eq = bool(g.integers(0, 2))
        dims = [n] * m if eq else [max(1, int(n * g.uniform(0.3, 1.0))) for _ in range(m)]
        probs.append(wl.random_problem(9800 + i, m, dims, eq, complex_=False, want_alpha=bool(g.integers(0, 2))))
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
