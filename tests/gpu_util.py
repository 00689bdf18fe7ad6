"""Helpers shared by the GPU parity tests (no product arithmetic here)."""
import numpy as np
import torch

import oracle

TOL = {torch.complex128: 1e-12, torch.float64: 1e-12, torch.complex64: 1e-4, torch.float32: 1e-4}
REAL_OF = {torch.complex64: torch.float32, torch.complex128: torch.float64}


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype):
    """Host array -> device tensor of `dtype` (complex dtypes keep the imaginary part)."""
    if a is None:
        return None
    a = np.asarray(a)
    if dtype.is_complex:
        t = torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128)))
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.real(a).astype(np.float64)))
    return t.to(dtype).to(dev())


def seen(a, dtype):
    """The exact values the GPU receives, as complex128 host data (oracle input)."""
    if a is None:
        return None
    t = to_dev(a, dtype).cpu()
    return t.to(torch.complex128).numpy()


def host(t):
    return None if t is None else t.detach().cpu().to(torch.complex128).numpy()


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_alpha(a, ao, dtype, what="", tol=None):
    """Scalar alpha = H x_1 ... x_m against the oracle: |a - ao| / |ao| within the
    same relative tolerance as the vector products."""
    tol = TOL[dtype] if tol is None else tol
    a, ao = complex(a), complex(ao)
    e = abs(a - ao) / max(abs(ao), 1e-300)
    assert e <= tol, f"alpha rel err {e:.3e} > {tol:g} {what}"
    return e


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def oracle_problem(prob, dtype):
    """Oracle result on exactly the inputs the GPU sees."""
    h = seen(prob.h, dtype)
    vecs = [seen(v, dtype) if v is not None else None for v in prob.vectors]
    if prob.is_block:
        return oracle.block_tvp(prob.m, prob.dims, prob.block_dims, h, vecs, prob.want_y, prob.want_alpha)
    return oracle.tvp(prob.m, prob.dims, h, vecs, prob.want_y, prob.want_alpha)
