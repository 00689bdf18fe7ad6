"""GPU batched forms: strided batches of one shape, and heterogeneous plans
(persistent task-queue kernel, one launch per pass, hipGraph replay) against
the oracle and against the plain single-product GPU path."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

from gpu_util import TOL, check_alpha, host, oracle_problem, print_case, rel, seen, to_dev  # noqa: E402


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64, torch.float64])
@pytest.mark.parametrize("m,n,B", [(3, 64, 7), (4, 1000, 3), (3, 3000, 4), (2, 10000, 2)])
def test_strided_batched_forward(dtype, m, n, B):
    import paper_1401_6238_amd as hk
    print_case(test="strided_forward", dtype=dtype, m=m, n=n, B=B)
    probs = [wl.random_problem(7000 + b, m, [n] * m, True, complex_=dtype.is_complex, want_alpha=True)
             for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.hankel_tvp_strided_batched(H, X, m, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        yo, ao = oracle_problem(p, dtype)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        ab = complex(host(a[b:b + 1])[0])
        check_alpha(ab, ao, dtype)


def test_block_strided_batched():
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    m, nb, B = 3, 40, 3
    probs = [wl.random_problem(7100 + b, m, [nb] * m, True, want_alpha=True, block_dims=[nb] * m) for b in range(B)]
    H = torch.stack([to_dev(p.h, dtype) for p in probs])
    X = torch.stack([to_dev(p.vectors[1], dtype) for p in probs])
    y, a = hk.block_hankel_tvp_strided_batched(H, X, m, nb, nb, True, True)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        yo, ao = oracle_problem(p, dtype)
        assert rel(host(y[b]), yo) <= TOL[dtype]
        check_alpha(complex(host(a[b:b + 1])[0]), ao, dtype)


def mixed_problems(seed, count):
    """Mixed orders, sizes (resident and 3-pass), equal/distinct vectors, some BHHB, some scalars."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        kind = g.integers(0, 10)
        m = int(g.integers(2, 6))
        if kind == 0:
            dims = [int(g.integers(2, 12)) for _ in range(m)]
            bd = [int(g.integers(2, 12)) for _ in range(m)]
            p = wl.random_problem(seed * 100 + i, m, dims, False, want_alpha=bool(g.integers(0, 2)), block_dims=bd)
        else:
            n = int(np.exp(g.uniform(np.log(2), np.log(3000))))
            eq = bool(g.integers(0, 2))
            dims = [n] * m if eq else [max(1, int(n * g.uniform(0.3, 1.0))) for _ in range(m)]
            p = wl.random_problem(seed * 100 + i, m, dims, eq, want_alpha=bool(g.integers(0, 2)),
                                  want_y=bool(g.integers(0, 4) > 0))
            if not p.want_y and not p.want_alpha:
                p.want_y = True
        out.append(p)
    return out


def plan_inputs(probs, dtype):
    items = []
    for p in probs:
        h = to_dev(p.h, dtype)
        if p.equal:
            x = to_dev(p.vectors[1], dtype)
            vecs = [x if (k > 0 or p.want_alpha) else None for k in range(p.m)]
        else:
            vecs = [to_dev(v, dtype) if v is not None else None for v in p.vectors]
        d = {"m": p.m, "dims": p.dims, "h": h, "vectors": vecs, "want_y": p.want_y, "want_alpha": p.want_alpha}
        if p.is_block:
            d["block_dims"] = p.block_dims
        items.append(d)
    return items


def check_plan_outputs(probs, outs, dtype):
    for p, (y, a) in zip(probs, outs):
        yo, ao = oracle_problem(p, dtype)
        if p.want_y:
            assert rel(host(y), yo) <= TOL[dtype]
        if p.want_alpha:
            av = complex(host(a.reshape(1))[0])
            check_alpha(av, ao, dtype)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_kind_restricted_oneshot_batches(dtype):
    """hankel_mode_products_batched and block_hankel_tvp_batched (the one-shot
    C entry points for one product kind) against the oracle."""
    import paper_1401_6238_amd as hk
    probs = mixed_problems(4242, 40)
    one_d = [p for p in probs if not p.is_block]
    blocks = [wl.random_problem(4300 + i, m, [n] * m, i % 2 == 0, want_alpha=True, block_dims=[nb] * m)
              for i, (m, n, nb) in enumerate([(3, 20, 15), (2, 33, 40), (4, 9, 12), (3, 64, 64)])]
    print_case(test="kind_batches", dtype=dtype, n1d=len(one_d), nblock=len(blocks))
    outs = hk.hankel_mode_products_batched(plan_inputs(one_d, dtype))
    torch.cuda.synchronize()
    check_plan_outputs(one_d, outs, dtype)
    outs = hk.block_hankel_tvp_batched(plan_inputs(blocks, dtype))
    torch.cuda.synchronize()
    check_plan_outputs(blocks, outs, dtype)


@pytest.mark.parametrize("flags", ["persistent", "multikernel"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_plan_mixed(flags, dtype):
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    print_case(test="plan_mixed", flags=flags, dtype=dtype)
    probs = mixed_problems(31, 60)
    f = _lib.HK_PLAN_PERSISTENT if flags == "persistent" else _lib.HK_PLAN_MULTIKERNEL
    plan = hk.Plan(plan_inputs(probs, dtype), flags=f)
    outs = plan.execute()
    plan.status()
    check_plan_outputs(probs, outs, dtype)
    first = [(host(y) if y is not None else None) for y, _ in outs]
    outs2 = plan.execute()
    plan.status()
    for a, (y, _) in zip(first, outs2):
        if a is not None:
            assert np.array_equal(a, host(y)), "repeated execution must be bitwise identical"
    plan.close()


def test_plan_matches_plain_path():
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    probs = mixed_problems(32, 25)
    items = plan_inputs(probs, dtype)
    plan = hk.Plan(items)
    outs = plan.execute()
    plan.status()
    for p, it, (y, a) in zip(probs, items, outs):
        if p.is_block:
            y2, a2 = hk.block_hankel_tvp(it["h"], it["vectors"], p.dims, p.block_dims, p.want_y, p.want_alpha)
        else:
            y2, a2 = hk.hankel_mode_products(it["h"], it["vectors"], p.dims, p.want_y, p.want_alpha)
        # the plan and the plain path, each against the oracle
        yo, ao = oracle_problem(p, dtype)
        if p.want_y:
            assert rel(host(y), yo) <= TOL[dtype]
            assert rel(host(y2), yo) <= TOL[dtype]
        if p.want_alpha:
            for aa in (a, a2):
                check_alpha(complex(host(aa.reshape(1))[0]), ao, dtype)
    plan.close()


@pytest.mark.parametrize("mode", ["persistent", "grouped"])
def test_plan_graph_replays(mode):
    """Graph replays with eager work in between; every replay checked.  The
    grouped plan's graph holds its launches on several streams (forked and
    joined per phase)."""
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    dtype = torch.complex64
    print_case(test="plan_graph_replays", mode=mode)
    probs = mixed_problems(33, 30)
    items = plan_inputs(probs, dtype)
    s = torch.cuda.Stream()
    base = _lib.HK_PLAN_PERSISTENT if mode == "persistent" else _lib.HK_PLAN_MULTIKERNEL
    with torch.cuda.stream(s):
        plan = hk.Plan(items, flags=base | _lib.HK_PLAN_GRAPH)
        for rep in range(3):
            for y, a in plan.outputs:
                if y is not None:
                    y.fill_(float("nan"))
            outs = plan.execute()
            plan.status()
            check_plan_outputs(probs, outs, dtype)
            junk = torch.randn(1 << 20, device="cuda") * 2  # unrelated eager work between replays
            torch.cuda.synchronize()
            del junk
    plan.close()


def test_one_shot_batched():
    import paper_1401_6238_amd as hk
    dtype = torch.complex128
    probs = mixed_problems(34, 12)
    outs = hk.hankel_tvp_batched(plan_inputs(probs, dtype))
    check_plan_outputs(probs, outs, dtype)


def test_mixed_batch_subset():
    """The first 48 instances of the 4096-problem mixed batch (m in {3,4,5}, n in [64, 16384])."""
    import paper_1401_6238_amd as hk
    dtype = torch.complex64
    probs = [wl.mixed_instance(i) for i in range(48)]
    plan = hk.Plan(plan_inputs(probs, dtype))
    outs = plan.execute()
    plan.status()
    check_plan_outputs(probs, outs, dtype)
    plan.close()


def test_persistent_barrier_timeout_path():
    """The bounded wait of the persistent schedule's grid barrier: with a bound
    of zero polls the kernel takes its error path (sets the error word and
    runs to its end), hk_plan_status reports it, and a plan with the default
    bound afterwards is correct again."""
    import paper_1401_6238_amd as hk
    from paper_1401_6238_amd import _lib
    dtype = torch.complex64
    probs = mixed_problems(33, 40)
    print_case(test="persistent_barrier_timeout")
    plan = hk.Plan(plan_inputs(probs, dtype), flags=_lib.HK_PLAN_PERSISTENT)
    plan.set_wait_bound(0)
    plan.execute()
    with pytest.raises(_lib.HankelError) as ei:
        plan.status()
    assert ei.value.code == 8  # HK_ERR_DEVICE_FAULT
    plan.close()
    plan = hk.Plan(plan_inputs(probs, dtype), flags=_lib.HK_PLAN_PERSISTENT)
    outs = plan.execute()
    plan.status()
    check_plan_outputs(probs, outs, dtype)
    plan.close()
