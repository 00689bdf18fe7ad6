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

from gpu_util import TOL, check_alpha, host, print_case, rel, seen, to_dev  # noqa: E402

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
        check_alpha(complex(host(a.reshape(1))[0]), ao, dtype, sched)


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
        check_alpha(complex(host(a.reshape(1))[0]), ao, dtype, sched)


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


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_odd_length_schedules(tmp_path, dtype):
    """The 3-pass path on N = 3 * 2^12 under a sweep of schedules (row split,
    rows per workgroup, rows in turn, column tiles, XCD numbering)."""
    import paper_1401_6238_amd as hk
    m, n = 3, 4096  # d_H = 12286, N = 3 * 4096
    hk.hk_set_fft_lengths("smallest")
    try:
        prob = wl.random_problem(4343, m, [n] * m, True, want_alpha=True)
        h, x = to_dev(prob.h, dtype), to_dev(prob.vectors[1], dtype)
        yo, ao = oracle.tvp(m, [n] * m, seen(prob.h, dtype), [seen(prob.vectors[1], dtype)] * m, True, True)
        key = (DT_CODE[dtype], 0, 0, 3, 12, -1, 0)
        for sched in [(4, 1, 8, 8, 0, 0, 1), (4, 2, 16, 4, -1, 1, 2), (4, 1, 16, 16, 1, 0, 4), (4, 4, 8, 1, 0, 1, 1),
                      (4, 1, 8, 16, -1, 0, 2)]:
            print_case(test="odd_schedules", dtype=dtype, sched=sched)
            install(tmp_path, key, sched)
            y, a = hk.hankel_tvp(h, x, m, True, True)
            torch.cuda.synchronize()
            assert rel(host(y), yo) <= TOL[dtype], sched
            check_alpha(complex(host(a.reshape(1))[0]), ao, dtype, sched)
    finally:
        hk.hk_set_fft_lengths("auto")


def test_autotuned_odd_and_real_shapes():
    """The autotuner on an odd-length strided batch and on a 3-pass real-input
    product; the tuned schedules give the oracle's results."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    m, n, B = 3, 4096, 16  # 16 x 2^14 >= 2^18: the default policy takes N = 3 * 2^12
    print_case(test="autotune_odd_real")
    hk.hk_autotune(dtype, "forward", m, n, batch=B)
    probs = [wl.random_problem(4400 + b, m, [n] * m, True, want_alpha=True) for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs[:3]):
        yo, ao = oracle.tvp(m, [n] * m, seen(p.h, dtype), [seen(p.vectors[1], dtype)] * m, True, True)
        assert rel(host(y[b]), yo) <= TOL[dtype]
    rdt = torch.float32
    m, n = 3, 5000  # real N = 16384: three passes on mirrored row pairs
    hk.hk_autotune(rdt, "forward", m, n)
    p = wl.random_problem(4500, m, [n] * m, True, complex_=False, want_alpha=True)
    y, a = hk.hankel_tvp(to_dev(p.h, rdt), to_dev(p.vectors[1], rdt), m, True, True)
    torch.cuda.synchronize()
    yo, ao = oracle.tvp(m, [n] * m, seen(p.h, rdt), [seen(p.vectors[1], rdt)] * m, True, True)
    assert rel(host(y), yo) <= TOL[rdt]
    check_alpha(complex(host(a.reshape(1))[0]), ao, rdt)


@pytest.mark.parametrize("rows", [1, 3, 5])
def test_ragged_workgroup_sums(tmp_path, rows):
    """Row-pass workgroups whose lane count is not a power of two (3 or 5
    rows per workgroup): the scalar's per-workgroup partial sums on the
    odd-factor rows (N = 3 * 2^12, complex, 16 lanes a row) and on the
    mirrored real row pairs (real N = 2^14, 32 lanes a pair), y and alpha
    against the oracle."""
    import paper_1401_6238_amd as hk
    hk.hk_set_fft_lengths("smallest")
    try:
        m, n = 3, 4096
        dtype = torch.complex64
        prob = wl.random_problem(4600 + rows, m, [n] * m, True, want_alpha=True)
        yo, ao = oracle.tvp(m, [n] * m, seen(prob.h, dtype), [seen(prob.vectors[1], dtype)] * m, True, True)
        print_case(test="ragged_sums_odd", rows=rows)
        install(tmp_path, (0, 0, 0, 3, 12, -1, 0), (4, rows, 8, 8, 0, 0, 1))
        y, a = hk.hankel_tvp(to_dev(prob.h, dtype), to_dev(prob.vectors[1], dtype), m, True, True)
        torch.cuda.synchronize()
        assert rel(host(y), yo) <= TOL[dtype]
        check_alpha(complex(host(a.reshape(1))[0]), ao, dtype, rows)
    finally:
        hk.hk_set_fft_lengths("auto")
    rdt = torch.float32
    m, n = 3, 5000  # real N = 2^14: rows of 2^7 complex points in mirrored pairs
    p = wl.random_problem(4700 + rows, m, [n] * m, True, complex_=False, want_alpha=True)
    yo, ao = oracle.tvp(m, [n] * m, seen(p.h, rdt), [seen(p.vectors[1], rdt)] * m, True, True)
    print_case(test="ragged_sums_real", rows=rows)
    install(tmp_path, (2, 0, 0, 2, 13, -1, 0), (8, rows, 16, 8, 0, 0, 1))
    y, a = hk.hankel_tvp(to_dev(p.h, rdt), to_dev(p.vectors[1], rdt), m, True, True)
    torch.cuda.synchronize()
    assert rel(host(y), yo) <= TOL[rdt]
    check_alpha(complex(host(a.reshape(1))[0]), ao, rdt, rows)


def test_factor5_schedules(tmp_path):
    """The three-pass length 5 * 2^12 (float) under schedules that run the
    factor-5 rows one per lane group (no rows in turn: 1 or 3 rows per
    workgroup) and streamed (2 or 4 rows in turn, split -1 / +1)."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    m, n = 3, 6500  # d_H = 19,498 -> 5 * 2^12 under the smallest-length policy
    hk.hk_set_fft_lengths("smallest")
    try:
        assert hk.hk_fft_layout(m * (n - 1) + 1)[0] == 5 << 12
        prob = wl.random_problem(4800, m, [n] * m, True, want_alpha=True)
        h, x = to_dev(prob.h, dtype), to_dev(prob.vectors[1], dtype)
        yo, ao = oracle.tvp(m, [n] * m, seen(prob.h, dtype), [seen(prob.vectors[1], dtype)] * m, True, True)
        for sched in [(4, 1, 8, 8, 0, 0, 1), (4, 3, 16, 16, 0, 0, 1), (4, 2, 8, 8, 0, 0, 2), (4, 1, 16, 4, 1, 1, 4),
                      (4, 2, 16, 8, -1, 0, 1)]:
            print_case(test="factor5_schedules", sched=sched)
            install(tmp_path, (0, 0, 0, 5, 12, -1, 0), sched)
            y, a = hk.hankel_tvp(h, x, m, True, True)
            torch.cuda.synchronize()
            assert rel(host(y), yo) <= TOL[dtype], sched
            check_alpha(complex(host(a.reshape(1))[0]), ao, dtype, sched)
    finally:
        hk.hk_set_fft_lengths("auto")
