"""Every schedule gives the same products: the plain 3-pass path, the BHHB
path and the adjoint are run under a sweep of schedules (row/column split,
elements per lane, rows per workgroup, rows in turn, column-tile width, XCD
tile numbering)
installed through the schedule database, and each result is compared with
the CPU oracle."""
import itertools
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, host, print_case, rel, seen, to_dev  # noqa: E402

DT_CODE = {torch.complex64: 0, torch.complex128: 1}


def sweep():
    combos = list(itertools.product([8, 16], [1, 2], [8, 16], [1, 4, 16], [-1, 0, 1], [0, 1], [1, 2, 4]))
    g = np.random.Generator(np.random.PCG64(77))
    idx = g.choice(len(combos), 24, replace=False)
    return [combos[i] for i in sorted(idx)] + [(8, 1, 8, 8, 0, 0, 1), (8, 1, 16, 16, 1, 1, 2), (8, 2, 8, 4, 0, 1, 4)]


def install(tmp_path, key, sched):
    import paper_1401_6238_amd as hk
    er, rows, ec, tw, split, xcd, iters = sched
    path = tmp_path / "db.txt"
    path.write_text(" ".join(map(str, key)) + f" : {er} {rows} {ec} {tw} {split} {xcd} {iters}\n")
    assert hk.hk_tune_load(str(path)) == 1


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_plain_multipass_schedules(tmp_path, dtype):
    import paper_1401_6238_amd as hk
    m, n = 3, 3000  # d_H = 8998, N = 2^14: three passes
    prob = wl.random_problem(4242, m, [n] * m, True, want_alpha=True)
    h, x = to_dev(prob.h, dtype), to_dev(prob.vectors[1], dtype)
    yo, ao = oracle.tvp(m, [n] * m, seen(prob.h, dtype), [seen(prob.vectors[1], dtype)] * m, True, True)
    key = (DT_CODE[dtype], 0, 0, 14, -1, 0)
    for sched in sweep():
        print_case(test="plain_schedules", dtype=dtype, sched=sched)
        install(tmp_path, key, sched)
        y, a = hk.hankel_tvp(h, x, m, True, True)
        torch.cuda.synchronize()
        assert rel(host(y), yo) <= TOL[dtype], sched
        assert abs(complex(host(a.reshape(1))[0]) - ao) <= 10 * TOL[dtype] * abs(ao), sched


def test_block_schedules(tmp_path):
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    dims, bdims = [40, 23, 9], [17, 30, 12]  # grid 70 x 57 -> 2^7 x 2^6
    prob = wl.random_problem(4343, 3, dims, False, block_dims=bdims, want_alpha=True)
    H = to_dev(prob.h, dtype)
    vecs = [to_dev(v, dtype) for v in prob.vectors]
    yo, ao = oracle.block_tvp(3, dims, bdims, seen(prob.h, dtype), [seen(v, dtype) for v in prob.vectors],
                              True, True)
    key = (0, 0, 1, 13, 6, 0)
    for sched in sweep():
        if sched[4] != 0:
            continue  # the BHHB grid is not split
        print_case(test="block_schedules", sched=sched)
        install(tmp_path, key, sched)
        y, a = hk.block_hankel_tvp(H, vecs, dims, bdims, True, True)
        torch.cuda.synchronize()
        assert rel(host(y), yo) <= TOL[dtype], sched
        assert abs(complex(host(a.reshape(1))[0]) - ao) <= 10 * TOL[dtype] * abs(ao), sched


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_adjoint_schedules(tmp_path, dtype):
    import paper_1401_6238_amd as hk
    m, n = 4, 1500  # d_H = 5997, N = 2^13
    g = wl.rng_for(44, 0)
    h = wl.cn(g, m * (n - 1) + 1, 1.0)
    x = wl.cn(g, n, 1.0 / n)
    v = wl.cn(g, n, 1.0)
    phi = complex(wl.cn(g, 1, 1.0)[0])
    gxo, gho = oracle.tvp_backward(m, seen(h, dtype), seen(x, dtype), seen(v, dtype),
                                   complex(seen(np.array([phi]), dtype)[0]))
    hd, xd, vd = to_dev(h, dtype), to_dev(x, dtype), to_dev(v, dtype)
    pd = to_dev(np.array([phi]), dtype)
    key = (DT_CODE[dtype], 1, 0, 13, -1, 0)
    for sched in sweep():
        print_case(test="adjoint_schedules", dtype=dtype, sched=sched)
        install(tmp_path, key, sched)
        gx, gh = hk.hankel_tvp_backward(hd, xd, m, vd, pd)
        torch.cuda.synchronize()
        assert rel(host(gx), gxo) <= TOL[dtype], sched
        assert rel(host(gh), gho) <= TOL[dtype], sched
