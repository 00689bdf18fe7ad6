"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned plain path, strided batches, persistent plans).

Expected values come from the CPU oracle through tests/golden/make_golden.py
(sampled outputs; the oracle's direct sums are too slow to run here), and
from closed forms that hold at any size (Vandermonde generating vectors,
Section 4.1 / 4.3), which check every output.
"""
import functools
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, print_case, rel, to_dev  # noqa: E402

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLD, f"{name}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (python tests/golden/make_golden.py)")
    return np.load(path)


def fingerprint(a):
    a = np.asarray(a, np.complex128)
    return np.array([a.real.sum(), a.imag.sum(), np.abs(a).sum()])


def same_inputs(fp_stored, arr):
    assert np.allclose(fp_stored, fingerprint(arr), rtol=1e-12, atol=1e-9), "generator drift"


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_large_single_golden(dtype):
    import paper_1401_6238_amd as hk
    g = golden("large_single")
    tag = "c128" if dtype == torch.complex128 else "c64"
    print_case(test="large_golden", dtype=tag)
    p = wl.large_single(0)
    same_inputs(g["large_fp_h"], p.h)
    same_inputs(g["large_fp_x"], p.vectors[1])
    hk.hk_autotune_tvp(dtype, 4, p.dims[0])
    y, a = hk.hankel_tvp(to_dev(p.h, dtype), to_dev(p.vectors[1], dtype), 4, True, True)
    torch.cuda.synchronize()
    idx = g["large_idx"]
    e = rel(host(y)[idx], g[f"large_{tag}_y"])
    ao = complex(g[f"large_{tag}_alpha"][0])
    ea = abs(complex(host(a.reshape(1))[0]) - ao) / abs(ao)
    print(f"large {tag}: y rel err {e:.3e}, alpha rel err {ea:.3e}")
    assert e <= TOL[dtype]
    assert ea <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_large_single_warm_golden(dtype):
    """The same product with h^ stored once (hankel_spectrum) and reused: a
    single warm product and a strided batch of two, against the oracle's
    sampled outputs and scalar."""
    import paper_1401_6238_amd as hk
    g = golden("large_single")
    tag = "c128" if dtype == torch.complex128 else "c64"
    print_case(test="large_warm_golden", dtype=tag)
    p = wl.large_single(0)
    same_inputs(g["large_fp_h"], p.h)
    same_inputs(g["large_fp_x"], p.vectors[1])
    n = p.dims[0]
    x = to_dev(p.vectors[1], dtype)
    hs = hk.hankel_spectrum(to_dev(p.h, dtype), 4, [n] * 4, -1)
    y, a = hk.hankel_mode_products_spectral(hs, 4, [n] * 4, [x] * 4, None, True, True)
    Y, A = hk.hankel_tvp_spectral_strided_batched(hs, torch.stack([x, x]), 4, True, True)
    torch.cuda.synchronize()
    idx = g["large_idx"]
    ao = complex(g[f"large_{tag}_alpha"][0])
    for yy, aa in ((host(y), complex(host(a.reshape(1))[0])), (host(Y[0]), complex(host(A[0:1])[0])),
                   (host(Y[1]), complex(host(A[1:2])[0]))):
        e = rel(yy[idx], g[f"large_{tag}_y"])
        ea = abs(aa - ao) / abs(ao)
        print(f"large warm {tag}: y rel err {e:.3e}, alpha rel err {ea:.3e}")
        assert e <= TOL[dtype]
        assert ea <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_shared_h_batch_golden(dtype):
    """A strided batch of 16 vectors sharing one stored h^ at the adjoint-batch
    shape (m = 4, n = 2^16, N = 2^18; the batch schedule of that shape, rows in
    turn): every instance is instance 0 of that workload, against the oracle's
    sampled forward outputs and scalar, and all 16 bit for bit alike."""
    import paper_1401_6238_amd as hk
    g = golden("adjoint_batch")
    tag = "c128" if dtype == torch.complex128 else "c64"
    print_case(test="shared_h_batch", dtype=tag)
    d = wl.adjoint_instance(0)
    same_inputs(g["adjoint_0_fp_h"], d["h"])
    n = d["n"]
    hs = hk.hankel_spectrum(to_dev(d["h"], dtype), 4, [n] * 4, -1)
    x = to_dev(d["x"], dtype)
    Y, A = hk.hankel_tvp_spectral_strided_batched(hs, x.expand(16, n).contiguous(), 4, True, True)
    torch.cuda.synchronize()
    idx = g["adjoint_0_idx_x"]
    fo = complex(g[f"adjoint_0_{tag}_f"][0])
    y0 = host(Y[0])
    e = rel(y0[idx], g[f"adjoint_0_{tag}_g"])
    ea = abs(complex(host(A[0:1])[0]) - fo) / abs(fo)
    print(f"shared-h batch {tag}: y rel err {e:.3e}, alpha rel err {ea:.3e}")
    assert e <= TOL[dtype] and ea <= TOL[dtype]
    for b in range(1, 16):
        assert np.array_equal(host(Y[b]), y0)


def test_large_single_vandermonde_all_outputs():
    """Noise-free twin of the large single-product input: every output against the closed form.

    FP64 only: rounding h to complex64 would perturb the exponential sum by
    more than the closed form can account for (the complex64 path is checked
    against the oracle on its rounded inputs above)."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    print_case(test="large_vandermonde", dtype=dtype)
    p = wl.large_single(0, sigma=0.0)
    params = p.meta["expsum"]
    n = p.dims[0]
    x = p.vectors[1]
    xs = np.asarray(x, np.complex128)
    y_cf = np.zeros(n, np.clongdouble)
    a_cf = np.clongdouble(0)
    for j in range(len(params.a)):
        zp = wl.powers_ld(params.z[j], n)
        s = np.sum(np.asarray(xs, np.clongdouble) * zp)
        y_cf += np.clongdouble(params.a[j]) * s ** 3 * zp
        a_cf += np.clongdouble(params.a[j]) * s ** 4
    y, a = hk.hankel_tvp(to_dev(p.h, dtype), to_dev(x, dtype), 4, True, True)
    e = rel(host(y), y_cf.astype(np.complex128))
    ea = abs(complex(host(a.reshape(1))[0]) - complex(a_cf)) / abs(complex(a_cf))
    print(f"vandermonde {dtype}: y {e:.3e} alpha {ea:.3e}")
    assert e <= TOL[dtype]
    assert ea <= TOL[dtype]


@pytest.mark.parametrize("flags", ["persistent", "grouped", "grouped_autotune"])
def test_mixed_batch_all_instances(flags):
    """All 4096 mixed instances in one plan, sampled outputs against the oracle
    (autotune: the plan the first execute's tuner keeps, executed twice)."""
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    g = golden("mixed_batch")
    print_case(test="mixed_batch", flags=flags)
    dtype = torch.complex64
    items, probs = [], []
    for i in range(4096):
        p = wl.mixed_instance(i)
        probs.append(p)
        h = to_dev(p.h, dtype)
        if p.equal:
            x = to_dev(p.vectors[1], dtype)
            vecs = [None] + [x] * (p.m - 1)
        else:
            vecs = [None] + [to_dev(v, dtype) for v in p.vectors[1:]]
        items.append({"m": p.m, "dims": p.dims, "h": h, "vectors": vecs})
    same_inputs(g["mixed_fp_h"][0], probs[0].h)
    same_inputs(g["mixed_fp_h"][4095], probs[4095].h)
    f = _lib.HK_PLAN_PERSISTENT if flags == "persistent" else _lib.HK_PLAN_MULTIKERNEL
    if flags == "grouped_autotune":
        f |= _lib.HK_PLAN_AUTOTUNE
    plan = hk.Plan(items, flags=f)
    outs = plan.execute()
    if flags == "grouped_autotune":
        t0, t1, mask = plan.tune_times()
        print(f"autotune: default {t0:.3f} ms, kept {t1:.3f} ms, power-of-two buckets {mask:#x}")
        assert 0.0 < t1 <= t0
        outs = plan.execute()
    plan.status()
    off, idx, ys = g["mixed_off"], g["mixed_idx"], g["mixed_y"]
    worst = 0.0
    for i in range(4096):
        sl = slice(off[i], off[i + 1])
        e = rel(host(outs[i][0])[idx[sl]], ys[sl])
        worst = max(worst, e)
    plan.close()
    print(f"mixed worst instance rel err {worst:.3e}")
    assert worst <= TOL[dtype]


@functools.lru_cache(maxsize=None)
def _instances(kind, count):
    make = wl.adjoint_instance if kind == "adjoint" else wl.block_instance
    with ThreadPoolExecutor(max_workers=16) as ex:
        return tuple(ex.map(make, range(count)))


def _scalar_invariant(x, y, f, dtype):
    """alpha = x_1^T (H x_2 ... x_m) (Section 3): the scalar equals the vector
    product dotted with the first vector, at any size.  Both sides come from the
    GPU: with ||dy|| <= tol ||y|| and |df| <= tol |f| <= tol ||x|| ||y||
    (Cauchy-Schwarz), |f - x^T y| <= 2 tol ||x|| ||y||."""
    x = np.asarray(x, np.complex128)
    y = np.asarray(y, np.complex128)
    ref = complex(np.dot(x, y))
    bound = 2 * TOL[dtype] * np.linalg.norm(x) * np.linalg.norm(y)
    assert abs(complex(f) - ref) <= bound, (complex(f), ref, bound)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_adjoint_batch_forward_and_adjoint(dtype):
    """Batch of 256 distinct instances (m=4, n=2^16), as the benchmark times it:
    forward g, f and the gradients of twelve instances against the oracle's
    sampled values, the scalar of every instance against x^T g."""
    import paper_1401_6238_amd as hk
    g = golden("adjoint_batch")
    tag = "c128" if dtype == torch.complex128 else "c64"
    print_case(test="adjoint_batch", dtype=tag)
    insts = [int(i) for i in g["adjoint_instances"]]
    data = _instances("adjoint", 256)
    for i in insts:
        same_inputs(g[f"adjoint_{i}_fp_h"], data[i]["h"])
    H = torch.stack([to_dev(d["h"], dtype) for d in data])
    X = torch.stack([to_dev(d["x"], dtype) for d in data])
    V = torch.stack([to_dev(d["v"], dtype) for d in data])
    PHI = to_dev(np.array([d["phi"] for d in data]), dtype)
    gy, f = hk.hankel_tvp_strided_batched(H, X, 4, True, True)
    gx, gh = hk.hankel_tvp_backward_strided_batched(H, X, 4, V, PHI)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    for i in insts:
        ix, ih = g[f"adjoint_{i}_idx_x"], g[f"adjoint_{i}_idx_h"]
        assert rel(host(gy[i])[ix], g[f"adjoint_{i}_{tag}_g"]) <= tol
        check_alpha(complex(host(f[i:i + 1])[0]), complex(g[f"adjoint_{i}_{tag}_f"][0]), dtype, i)
        assert rel(host(gx[i])[ix], g[f"adjoint_{i}_{tag}_gx"]) <= tol
        assert rel(host(gh[i])[ih], g[f"adjoint_{i}_{tag}_gh"]) <= tol
    Xh, Gh, Fh = host(X), host(gy), host(f)
    for b in range(256):
        _scalar_invariant(Xh[b], Gh[b], Fh[b], dtype)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_adjoint_batch_autograd(dtype):
    """The batch of 256 (m=4, n=2^16) through the autograd Function, whose
    forward keeps x^ and whose backward reuses it: g, f and the gradients of
    the twelve sampled instances against the oracle's values."""
    import paper_1401_6238_amd as hk
    g = golden("adjoint_batch")
    tag = "c128" if dtype == torch.complex128 else "c64"
    print_case(test="adjoint_batch_autograd", dtype=tag)
    insts = [int(i) for i in g["adjoint_instances"]]
    data = _instances("adjoint", 256)
    H = torch.stack([to_dev(d["h"], dtype) for d in data]).requires_grad_(True)
    X = torch.stack([to_dev(d["x"], dtype) for d in data]).requires_grad_(True)
    V = torch.stack([to_dev(d["v"], dtype) for d in data])
    PHI = to_dev(np.array([d["phi"] for d in data]), dtype)
    gy, f = hk.hankel_tvp_autograd(H, X, 4)
    gH, gX = torch.autograd.grad([gy, f], [H, X], [V, PHI])
    torch.cuda.synchronize()
    tol = TOL[dtype]
    for i in insts:
        ix, ih = g[f"adjoint_{i}_idx_x"], g[f"adjoint_{i}_idx_h"]
        assert rel(host(gy[i].detach())[ix], g[f"adjoint_{i}_{tag}_g"]) <= tol
        check_alpha(complex(host(f[i:i + 1].detach())[0]), complex(g[f"adjoint_{i}_{tag}_f"][0]), dtype, i)
        assert rel(host(gX[i])[ix], g[f"adjoint_{i}_{tag}_gx"]) <= tol
        assert rel(host(gH[i])[ih], g[f"adjoint_{i}_{tag}_gh"]) <= tol


def test_block_batch():
    """64 distinct BHHB tensors (m=3, 512 blocks of 512, 2048^2 grid): sampled
    outputs of six tensors against the oracle, the scalar of every tensor
    against vec(X)^T vec(Y)."""
    import paper_1401_6238_amd as hk
    g = golden("block_batch")
    print_case(test="block_batch")
    dtype = torch.complex64
    insts = [int(i) for i in g["block_instances"]]
    data = _instances("block", 64)
    for i in insts:
        same_inputs(g[f"block_{i}_fp_h"], data[i].h)
    Hs = torch.stack([to_dev(d.h, dtype) for d in data])
    Xs = torch.stack([to_dev(d.vectors[1], dtype) for d in data])
    y, a = hk.block_hankel_tvp_strided_batched(Hs, Xs, 3, 512, 512, True, True)
    torch.cuda.synchronize()
    for i in insts:
        e = rel(host(y[i])[g[f"block_{i}_idx"]], g[f"block_{i}_y"])
        print(f"block tensor {i}: y {e:.3e}")
        assert e <= TOL[dtype]
        check_alpha(complex(host(a[i:i + 1])[0]), complex(g[f"block_{i}_alpha"][0]), dtype, i)
    Xh, Yh, Ah = host(Xs), host(y), host(a)
    for b in range(64):
        _scalar_invariant(Xh[b], Yh[b], Ah[b], dtype)


def test_block_level2_closed_form():
    """Noise-free twin of tensor 0: every output against the level-2 Vandermonde form."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    p = wl.block_instance(0, sigma=0.0)
    a_, z1, z2, _ = p.meta["expsum2"]
    nb = 512
    xs = p.vectors[1].reshape(nb, nb)  # [j, i]
    Y = np.zeros((nb, nb), np.clongdouble)
    alpha = np.clongdouble(0)
    for t in range(len(a_)):
        p1, p2 = wl.powers_ld(z1[t], nb), wl.powers_ld(z2[t], nb)
        s = np.sum(np.asarray(xs, np.clongdouble) * np.outer(p2, p1))
        Y += np.clongdouble(a_[t]) * s * s * np.outer(p2, p1)
        alpha += np.clongdouble(a_[t]) * s ** 3
    x = to_dev(p.vectors[1], dtype)
    y, a = hk.block_hankel_tvp(to_dev(p.h, dtype), [x] * 3, [nb] * 3, [nb] * 3, True, True)
    e = rel(host(y), Y.astype(np.complex128).ravel())
    ea = abs(complex(host(a.reshape(1))[0]) - complex(alpha)) / abs(complex(alpha))
    print(f"block closed form: y {e:.3e} alpha {ea:.3e}")
    assert e <= TOL[dtype] and ea <= TOL[dtype]
