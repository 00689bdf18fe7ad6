"""HOOI for square Hankel tensors (Algorithm 4.2) on the GPU against the
FP64 oracle: the randomized initial subspace against the dense SVD of the
Hankel matrix, and the iterations (same starting U) against the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402

PTOL = {torch.complex128: 1e-9, torch.complex64: 2e-3}


def signal(n, m, r, sigma, seed):
    g = wl.rng_for(60, seed)
    h, _ = wl.exp_sum_vector(g, m * (n - 1) + 1, r, sigma)
    return h


def proj_dist(U, V):
    U = np.asarray(U, np.complex128)
    V = np.asarray(V, np.complex128)
    return float(np.linalg.norm(U @ U.conj().T - V @ V.conj().T))


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("m,n,R", [(3, 64, 3), (4, 40, 2), (3, 700, 4)])
def test_hooi_matches_oracle(dtype, m, n, R):
    from paper_1401_6238_amd import hooi
    print_case(test="hooi", dtype=dtype, m=m, n=n, R=R)
    h = signal(n, m, R, 1e-3, 10 * m + n)
    hd = to_dev(h, dtype)
    hs = seen(h, dtype)
    U0o = oracle.hankel_leading_subspace(hs, n, R)
    U0g = hooi.hankel_leading_subspace(hd, n, R)
    assert proj_dist(host(U0g), U0o) <= PTOL[dtype]
    # iterations from the same start
    Uo, So = oracle.hooi(m, hs, R, iters=3, U0=U0o)
    Ug, Sg, hist = hooi.hooi(hd, m, R, iters=3, U0=to_dev(U0o.reshape(-1), dtype).reshape(n, R))
    torch.cuda.synchronize()
    assert proj_dist(host(Ug), Uo) <= PTOL[dtype]
    # the core S = H conj(U)^m element by element: the oracle's core of the GPU's
    # own U (the subspace agrees above; its basis is only fixed up to a rotation)
    _, So_g = oracle.hooi(m, hs, R, iters=0, U0=host(Ug))
    assert rel(host(Sg), So_g) <= TOL[dtype]
    assert len(hist) == 3
