"""Seeded synthetic inputs shaped like the paper's exponential-data-fitting signals.

This module only draws random numbers and lays them out; it holds none of the
Hankel tensor-vector product arithmetic.  Both the CPU oracle tests and the GPU
path draw their inputs from here, so the two sides always see the same data.

Signal model (Section 4.1, 1D exponential model; Section 4.3, 2D model):
the generating vector of a Hankel tensor built from a signal is the signal
itself, ``h_k = sum_j a_j z_j^k`` with poles ``z_j = exp(-alpha_j + i omega_j)``
(sampling interval 1), optionally plus circular complex Gaussian noise.  The 2D
generating matrix is ``H[k1, k2] = sum_j a_j z1_j^k1 z2_j^k2``.

Powers ``z^k`` are accumulated by a sequential product in 80-bit extended
precision, so that the stored double values equal the exact powers of the
stored double pole to ~1e-14 relative even at k ~ 1e6; closed-form checks built
on the returned ``(a, z)`` are then meaningful at FP64 tolerances.

Reading of "CN(0, s^2)": real and imaginary parts are i.i.d. N(0, s^2 / 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 14016238


# one seed stream per workload family
STREAM_SMALL_REAL, STREAM_LARGE_SINGLE, STREAM_MIXED, STREAM_ADJOINT, STREAM_BLOCK = 1, 2, 3, 4, 5


def rng_for(stream: int, instance: int = 0) -> np.random.Generator:
    """Counter-style seeding: one independent PCG64 stream per (workload family, instance)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * stream + instance))


def cn(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    """Circular complex Gaussian CN(0, var) samples (complex128)."""
    s = math.sqrt(var / 2.0)
    return (rng.standard_normal(shape) * s + 1j * rng.standard_normal(shape) * s).astype(np.complex128)


def powers(z: complex, count: int) -> np.ndarray:
    """z^0 .. z^(count-1) as complex128, accumulated in extended precision."""
    if count <= 0:
        return np.zeros(0, np.complex128)
    seq = np.full(count, np.clongdouble(z), dtype=np.clongdouble)
    seq[0] = 1
    return np.cumprod(seq).astype(np.complex128)


def powers_ld(z: complex, count: int) -> np.ndarray:
    """Same as :func:`powers` but kept in extended precision (for closed forms)."""
    if count <= 0:
        return np.zeros(0, np.clongdouble)
    seq = np.full(count, np.clongdouble(z), dtype=np.clongdouble)
    seq[0] = 1
    return np.cumprod(seq)


@dataclass
class ExpSum:
    """Parameters of an exponential sum h_k = sum_j a_j z_j^k (+ noise)."""
    a: np.ndarray  # complex128 amplitudes
    z: np.ndarray  # complex128 poles
    sigma: float


def exp_sum_vector(rng: np.random.Generator, d: int, r: int, sigma: float,
                   alpha_range=(1e-6, 1e-4), omega_range=(0.0, math.pi)):
    """1D generating vector of length d: r damped sinusoids plus CN(0, sigma^2) noise."""
    a = cn(rng, r, 1.0)
    alpha = rng.uniform(alpha_range[0], alpha_range[1], r)
    omega = rng.uniform(omega_range[0], omega_range[1], r)
    z = np.exp(-alpha + 1j * omega).astype(np.complex128)
    acc = np.zeros(d, np.clongdouble)
    for j in range(r):
        acc += np.clongdouble(a[j]) * powers_ld(z[j], d)
    h = acc.astype(np.complex128)
    if sigma > 0:
        h = h + cn(rng, d, sigma * sigma)
    return h, ExpSum(a, z, sigma)


def exp_sum_matrix(rng: np.random.Generator, rows: int, cols: int, r: int, sigma: float,
                   mag_range=(1e-5, 1e-3), arg_range=(0.0, math.pi)):
    """2D generating matrix (rows x cols), returned column-major as a flat vector.

    H[k1, k2] = sum_j a_j z1_j^k1 z2_j^k2 (+ noise); |z| = exp(-U[mag_range]),
    arg z ~ U[arg_range].  Flat index is k1 + rows * k2.
    """
    a = cn(rng, r, 1.0)
    z1 = np.exp(-rng.uniform(*mag_range, r) + 1j * rng.uniform(*arg_range, r)).astype(np.complex128)
    z2 = np.exp(-rng.uniform(*mag_range, r) + 1j * rng.uniform(*arg_range, r)).astype(np.complex128)
    # [k2, k1] so that ravel() is column-major in (k1, k2).  The powers are
    # accumulated in extended precision; the outer products (one rounding
    # each) are formed in double precision.
    acc = np.zeros((cols, rows), np.complex128)
    for j in range(r):
        p1 = powers(z1[j], rows)
        p2 = powers(z2[j], cols) * a[j]
        acc += np.outer(p2, p1)
    H = acc.ravel()
    if sigma > 0:
        H = H + cn(rng, rows * cols, sigma * sigma)
    return H, (a, z1, z2, sigma)


# ----------------------------------------------------------------------------
# Problem containers
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """One Hankel (or BHHB) tensor-vector product problem, host arrays.

    1D: tensor dims ``dims`` (n_1..n_m), generating vector ``h`` of length
    sum(dims) - m + 1.  ``vectors[p]`` multiplies mode p+1; ``vectors[0]`` is
    only used for the scalar product.  ``equal`` means every vector is the same
    array (H x^{m-1} / H x^m).
    BHHB: ``block_dims`` (N_1..N_m) are the numbers of blocks, ``dims`` the
    block sizes; ``h`` is the generating matrix, column-major, of shape
    (sum n_p - m + 1) x (sum N_p - m + 1); vector p has length n_p * N_p.
    """
    m: int
    dims: List[int]
    h: np.ndarray
    vectors: List[Optional[np.ndarray]]
    equal: bool
    want_y: bool = True
    want_alpha: bool = False
    block_dims: Optional[List[int]] = None
    meta: dict = field(default_factory=dict)

    @property
    def is_block(self) -> bool:
        return self.block_dims is not None

    @property
    def d_h(self) -> int:
        return sum(self.dims) - self.m + 1

    @property
    def out_len(self) -> int:
        if self.is_block:
            return self.dims[0] * self.block_dims[0]
        return self.dims[0]


def _real_or_complex(rng, n, real, var=1.0):
    if real:
        return rng.uniform(-1.0, 1.0, n)
    return cn(rng, n, var)


def small_real(instance: int = 0) -> Problem:
    """m=3, n=64 square Hankel tensor, real float64 U[-1,1] inputs; y = H x^2 and H x^3."""
    g = rng_for(STREAM_SMALL_REAL, instance)
    m, n = 3, 64
    d = m * (n - 1) + 1
    h = g.uniform(-1.0, 1.0, d)
    x = g.uniform(-1.0, 1.0, n)
    return Problem(m, [n] * m, h, [x] * m, True, True, True, meta={"workload": "small_real", "real": True})


def large_single(instance: int = 0, sigma: float = 1e-3, n: int = 1 << 18, r: int = 8) -> Problem:
    """m=4, n=2^18 square Hankel tensor; h an 8-term exponential sum + noise; x ~ CN(0, 1/n)."""
    g = rng_for(STREAM_LARGE_SINGLE, instance)
    m = 4
    d = m * (n - 1) + 1
    h, params = exp_sum_vector(g, d, r, sigma)
    x = cn(g, n, 1.0 / n)
    return Problem(m, [n] * m, h, [x] * m, True, True, True, meta={"workload": "large_single", "expsum": params})


def mixed_instance(instance: int) -> Problem:
    """One instance of the 4096-problem mixed batch (m in {3,4,5}, n log-uniform in [64, 16384])."""
    g = rng_for(STREAM_MIXED, instance)
    m = int(g.integers(3, 6))
    n = int(round(math.exp(g.uniform(math.log(64), math.log(16384)))))
    r = int(g.integers(2, 17))
    equal = bool(g.integers(0, 2))
    d = m * (n - 1) + 1
    h, params = exp_sum_vector(g, d, r, 1e-3)
    if equal:
        x = cn(g, n, 1.0 / n)
        vecs = [None] + [x] * (m - 1)
    else:
        vecs = [None] + [cn(g, n, 1.0 / n) for _ in range(m - 1)]
    return Problem(m, [n] * m, h, vecs, equal, True, False,
                   meta={"workload": "mixed", "expsum": params, "instance": instance})


def mixed_batch(count: int = 4096) -> List[Problem]:
    return [mixed_instance(i) for i in range(count)]


def adjoint_instance(instance: int, n: int = 1 << 16, sigma: float = 1e-3) -> dict:
    """m=4, n=2^16 forward (g = H x^3, f = H x^4) plus cotangents v ~ CN(0,1)^n, phi ~ CN(0,1)."""
    g = rng_for(STREAM_ADJOINT, instance)
    m = 4
    d = m * (n - 1) + 1
    h, params = exp_sum_vector(g, d, 8, sigma)
    x = cn(g, n, 1.0 / n)
    v = cn(g, n, 1.0)
    phi = complex(cn(g, 1, 1.0)[0])
    return {"m": m, "n": n, "h": h, "x": x, "v": v, "phi": phi, "expsum": params}


def block_instance(instance: int, nb: int = 512, sigma: float = 1e-3, r: int = 6,
                     m: int = 3) -> Problem:
    """BHHB order 3: block size n_p = 512, N_p = 512 blocks per mode; H is 1534 x 1534."""
    g = rng_for(STREAM_BLOCK, instance)
    dims = [nb] * m
    bdims = [nb] * m
    rows = sum(dims) - m + 1
    cols = sum(bdims) - m + 1
    H, params = exp_sum_matrix(g, rows, cols, r, sigma)
    x = cn(g, nb * nb, 1.0)
    return Problem(m, dims, H, [x] * m, True, True, True, block_dims=bdims,
                   meta={"workload": "block", "expsum2": params, "instance": instance})


def random_problem(seed: int, m: int, dims, equal: bool, complex_: bool = True,
                   want_y: bool = True, want_alpha: bool = False, block_dims=None,
                   integer: Optional[int] = None) -> Problem:
    """Generic seeded problem for parity / edge-case tests.

    ``integer=k`` draws integer entries in [-k, k] (real and imaginary parts when
    complex) so that exact results fit in int64 and in the FP64 mantissa.
    """
    g = np.random.Generator(np.random.PCG64(SEED_BASE + 7 * 1000003 + seed))
    dims = list(dims)
    if block_dims is None:
        d = sum(dims) - m + 1
        lens = dims
    else:
        block_dims = list(block_dims)
        d = (sum(dims) - m + 1) * (sum(block_dims) - m + 1)
        lens = [dims[p] * block_dims[p] for p in range(m)]

    def draw(n, var=1.0):
        if integer is not None:
            re = g.integers(-integer, integer + 1, n).astype(np.float64)
            if not complex_:
                return re
            im = g.integers(-integer, integer + 1, n).astype(np.float64)
            return re + 1j * im
        if complex_:
            return cn(g, n, var)
        return g.uniform(-1.0, 1.0, n)

    h = draw(d)
    if equal:
        if len(set(lens)) != 1:
            raise ValueError("equal vectors need equal mode lengths")
        x = draw(lens[0], 1.0 / max(lens[0], 1))
        vecs = [x] * m
    else:
        vecs = [draw(lens[p], 1.0 / max(lens[p], 1)) for p in range(m)]
    if not want_alpha:
        vecs = [None] + vecs[1:]
    return Problem(m, dims, h, vecs, equal, want_y, want_alpha, block_dims=block_dims,
                   meta={"seed": seed})
