"""Hankel tensor-matrix products H x_2 U ... x_m U (Section 4.2) on the GPU
against the oracle (columns are tensor-vector products), including the
symmetric completion of the columns and a multipass size."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402


@pytest.mark.parametrize("m,n,R,dtype", [
    (3, 40, 3, torch.complex128), (3, 40, 3, torch.complex64), (2, 50, 5, torch.complex128),
    (4, 30, 3, torch.float64), (3, 3000, 4, torch.complex64), (5, 12, 2, torch.complex128),
])
def test_tensor_matrix(m, n, R, dtype):
    import paper_1401_6238_amd as hk
    print_case(test="tensor_matrix", m=m, n=n, R=R, dtype=dtype)
    g = np.random.Generator(np.random.PCG64(900 + 10 * m + n + R))
    cplx = dtype.is_complex
    h = g.normal(size=m * (n - 1) + 1) + (1j * g.normal(size=m * (n - 1) + 1) if cplx else 0)
    U = g.normal(size=(n, R)) + (1j * g.normal(size=(n, R)) if cplx else 0)
    hd = to_dev(h, dtype)
    Ud = to_dev(U.reshape(-1), dtype).reshape(n, R)
    T = hk.hankel_tensor_matrix(hd, Ud, m)
    torch.cuda.synchronize()
    assert tuple(T.shape) == (n,) + (R,) * (m - 1)
    ref = oracle.tensor_matrix(m, seen(h, dtype), seen(U.reshape(-1), dtype).reshape(n, R))
    got = host(T.permute([0] + list(range(m - 1, 0, -1))).reshape(n, -1))  # (i, j_m, ..., j_2)
    assert rel(got, ref) <= TOL[dtype]
    # symmetric in the column indices, bit for bit (copied columns)
    if m >= 3 and R >= 2:
        t = host(T)
        assert np.array_equal(t[:, 0, 1], t[:, 1, 0]) if m == 3 else True
