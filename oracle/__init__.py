"""CPU oracle for the Hankel tensor-vector product -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it.

The arithmetic lives in ``hk_oracle.c`` (plain C, FP64 and complex int64, no
FFT): the Section 1 / Section 2.1 definition of the products, with the terms of
each output gathered by their index sum into direct convolutions followed by a
correlation with the generating vector.  This module only marshals numpy
arrays to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hk_oracle.c")
_LIB = os.path.join(_HERE, "libhk_oracle.so")
_lib_handle = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.hko_conv_range.argtypes = [P, I64, P, I64, I64, I64, P]
        lib.hko_conv.argtypes = [P, I64, P, I64, P]
        lib.hko_corr.argtypes = [P, I64, P, I64, I64, P]
        lib.hko_tvp.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.hko_tvp_sampled.argtypes = [ctypes.c_int, P, P, P, P, I64, P, P]
        lib.hko_tvp_i64.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.hko_block_tvp.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        lib.hko_block_tvp_i64.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        lib.hko_block_tvp_sampled.argtypes = [ctypes.c_int, P, P, P, P, P, I64, P, P]
        lib.hko_tvp_backward.argtypes = [ctypes.c_int, I64, P, P, P, P, P, P]
        lib.hko_mode_backward.argtypes = [ctypes.c_int, P, P, P, P, P, P, P]
        lib.hko_block_backward.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, P]
        lib.hko_dft_sampled.argtypes = [ctypes.c_int, P, I64, I64, P, I64, P]
        lib.hko_tvp_comp.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.hko_max_threads.argtypes = []
        lib.hko_set_threads.argtypes = [ctypes.c_int]
        for f in (lib.hko_conv_range, lib.hko_conv, lib.hko_corr, lib.hko_tvp, lib.hko_tvp_sampled,
                  lib.hko_tvp_i64, lib.hko_block_tvp, lib.hko_block_tvp_i64, lib.hko_block_tvp_sampled,
                  lib.hko_tvp_backward, lib.hko_mode_backward, lib.hko_block_backward, lib.hko_dft_sampled,
                  lib.hko_tvp_comp,
                  lib.hko_max_threads, lib.hko_set_threads):
            f.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def max_threads() -> int:
    return int(_lib().hko_max_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the previous count."""
    return int(_lib().hko_set_threads(int(n)))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _vec_ptrs(vectors: Sequence[Optional[np.ndarray]]):
    arr = (ctypes.c_void_p * len(vectors))()
    for i, v in enumerate(vectors):
        arr[i] = None if v is None else v.ctypes.data
    return arr


def conv(a, b, k0: int = 0, k1: Optional[int] = None) -> np.ndarray:
    """Linear convolution (a * b)_k for k in [k0, k1)."""
    a, b = _c128(a), _c128(b)
    if k1 is None:
        k1 = len(a) + len(b) - 1
    out = np.empty(max(k1 - k0, 0), np.complex128)
    _check(_lib().hko_conv_range(_ptr(a), len(a), _ptr(b), len(b), k0, k1, _ptr(out)), "conv")
    return out


def corr(h, w, ny: int) -> np.ndarray:
    """y_i = sum_k h_{i+k} w_k, i < ny."""
    h, w = _c128(h), _c128(w)
    out = np.empty(ny, np.complex128)
    _check(_lib().hko_corr(_ptr(h), len(h), _ptr(w), len(w), ny, _ptr(out)), "corr")
    return out


def _prep(m, dims, h, vectors, need_first):
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    if len(dims) != m:
        raise ValueError("dims must have m entries")
    h = _c128(h)
    vecs: List[Optional[np.ndarray]] = []
    for p in range(m):
        v = vectors[p] if p < len(vectors) else None
        if v is None:
            if p == 0 and not need_first:
                vecs.append(None)
                continue
            raise ValueError(f"vector {p + 1} is required")
        v = _c128(v)
        vecs.append(v)
    return dims, h, vecs


def tvp(m: int, dims, h, vectors, want_y: bool = True, want_alpha: bool = False, compensated: bool = False):
    """Returns (y, alpha): y = H x_2 ... x_m (length dims[0]), alpha = H x_1 ... x_m.
    compensated=True: every sum by the Dot2 algorithm (twice the working
    precision), to measure the rounding error of the default blocked sums."""
    dims, h, vecs = _prep(m, dims, h, vectors, want_alpha)
    y = np.empty(int(dims[0]), np.complex128) if want_y else None
    alpha = np.zeros(1, np.complex128) if want_alpha else None
    keep = _vec_ptrs(vecs)
    fn = _lib().hko_tvp_comp if compensated else _lib().hko_tvp
    _check(fn(m, _ptr(dims), _ptr(h), keep, _ptr(y), _ptr(alpha)), "tvp")
    return y, (None if alpha is None else complex(alpha[0]))


def tvp_sampled(m: int, dims, h, vectors, idx, want_alpha: bool = False):
    """y at the given output indices (and alpha if asked)."""
    dims, h, vecs = _prep(m, dims, h, vectors, want_alpha)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    y = np.empty(len(idx), np.complex128)
    alpha = np.zeros(1, np.complex128) if want_alpha else None
    keep = _vec_ptrs(vecs)
    _check(_lib().hko_tvp_sampled(m, _ptr(dims), _ptr(h), keep, _ptr(idx), len(idx), _ptr(y),
                                  _ptr(alpha)), "tvp_sampled")
    return y, (None if alpha is None else complex(alpha[0]))


def _i64pairs(a) -> np.ndarray:
    a = np.asarray(a)
    re = np.real(a)
    im = np.imag(a) if np.iscomplexobj(a) else np.zeros_like(re)
    if not (np.all(re == np.round(re)) and np.all(im == np.round(im))):
        raise ValueError("integer oracle needs integer-valued inputs")
    out = np.empty((len(a), 2), np.int64)
    out[:, 0] = re.astype(np.int64)
    out[:, 1] = im.astype(np.int64)
    return np.ascontiguousarray(out)


def tvp_i64(m: int, dims, h, vectors, want_y: bool = True, want_alpha: bool = False):
    """Exact complex-int64 product.  Returns (y, alpha) as (n,2)/(2,) int64 arrays."""
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    hi = _i64pairs(h)
    vecs = [None if (v is None) else _i64pairs(v) for v in vectors]
    y = np.empty((int(dims[0]), 2), np.int64) if want_y else None
    alpha = np.zeros(2, np.int64) if want_alpha else None
    keep = _vec_ptrs(vecs)
    _check(_lib().hko_tvp_i64(m, _ptr(dims), _ptr(hi), keep, _ptr(y), _ptr(alpha)), "tvp_i64")
    return y, alpha


def block_tvp(m: int, dims, block_dims, H, vectors, want_y: bool = True, want_alpha: bool = False):
    """BHHB product.  H column-major (sum n - m + 1) x (sum N - m + 1); y = vec(Y), Y n_1 x N_1."""
    dims, H, vecs = _prep(m, dims, H, vectors, want_alpha)
    bd = np.ascontiguousarray(np.asarray(block_dims, dtype=np.int64))
    y = np.empty(int(dims[0] * bd[0]), np.complex128) if want_y else None
    alpha = np.zeros(1, np.complex128) if want_alpha else None
    keep = _vec_ptrs(vecs)
    _check(_lib().hko_block_tvp(m, _ptr(dims), _ptr(bd), _ptr(H), keep, _ptr(y), _ptr(alpha)),
           "block_tvp")
    return y, (None if alpha is None else complex(alpha[0]))


def block_levels_tvp(m: int, dims, G, vectors, want_y: bool = True, want_alpha: bool = False):
    """Level-k block Hankel product (Section 2.2: a block Hankel tensor whose
    blocks are level-(k-1) block Hankel tensors), k = len(dims), in plain
    numpy FP64 with direct sums.

    dims[t][p] is the size of mode p at level t (t = 0 innermost); G is the
    generating tensor of size d_0 x ... x d_{k-1}, d_t = sum_p dims[t][p] - m + 1
    (flat column-major, or an array of that shape); vectors[p] = vec(X_p),
    column-major.  The entry of the level-k tensor at the multi-indices
    (i_1, ..., i_m) is G[i_1 + ... + i_m] (sums taken level by level), so,
    gathering terms by their index sum, W = X_2 * ... * X_m (k-dimensional
    linear convolutions) and Y[i] = sum_a G[i + a] W[a]; alpha = sum_s G[s]
    (X_1 * W)[s].  Returns (vec(Y) or None, alpha or None).
    """
    k = len(dims)
    d = [sum(int(v) for v in dims[t]) - m + 1 for t in range(k)]
    G = np.asarray(G, np.complex128).reshape(d, order="F")
    X = [None if v is None else np.asarray(v, np.complex128).reshape([int(dims[t][p]) for t in range(k)], order="F")
         for p, v in enumerate(vectors)]

    def conv(A, B):
        out = np.zeros([a + b - 1 for a, b in zip(A.shape, B.shape)], np.complex128)
        for idx in np.ndindex(*B.shape):
            out[tuple(slice(i, i + n) for i, n in zip(idx, A.shape))] += A * B[idx]
        return out

    W = X[1]
    for p in range(2, m):
        W = conv(W, X[p])
    y = None
    if want_y:
        n1 = [int(dims[t][0]) for t in range(k)]
        Y = np.zeros(n1, np.complex128)
        for idx in np.ndindex(*W.shape):
            Y += W[idx] * G[tuple(slice(i, i + n) for i, n in zip(idx, n1))]
        y = Y.reshape(-1, order="F")
    alpha = None
    if want_alpha:
        V = conv(X[0], W)
        alpha = complex(np.sum(G[tuple(slice(0, n) for n in V.shape)] * V))
    return y, alpha


def block_tvp_sampled(m: int, dims, block_dims, H, vectors, idx, want_alpha: bool = False):
    """BHHB product at flat output indices idx (column-major in the n_1 x N_1 result)."""
    dims, H, vecs = _prep(m, dims, H, vectors, want_alpha)
    bd = np.ascontiguousarray(np.asarray(block_dims, dtype=np.int64))
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    y = np.empty(len(idx), np.complex128)
    alpha = np.zeros(1, np.complex128) if want_alpha else None
    keep = _vec_ptrs(vecs)
    _check(_lib().hko_block_tvp_sampled(m, _ptr(dims), _ptr(bd), _ptr(H), keep, _ptr(idx), len(idx), _ptr(y),
                                        _ptr(alpha)), "block_tvp_sampled")
    return y, (None if alpha is None else complex(alpha[0]))


def block_tvp_i64(m: int, dims, block_dims, H, vectors, want_y: bool = True, want_alpha: bool = False):
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    bd = np.ascontiguousarray(np.asarray(block_dims, dtype=np.int64))
    Hi = _i64pairs(H)
    vecs = [None if (v is None) else _i64pairs(v) for v in vectors]
    y = np.empty((int(dims[0] * bd[0]), 2), np.int64) if want_y else None
    alpha = np.zeros(2, np.int64) if want_alpha else None
    keep = _vec_ptrs(vecs)
    _check(_lib().hko_block_tvp_i64(m, _ptr(dims), _ptr(bd), _ptr(Hi), keep, _ptr(y), _ptr(alpha)),
           "block_tvp_i64")
    return y, alpha


def tvp_backward(m: int, h, x, v=None, phi=None, want_grad_x: bool = True, want_grad_h: bool = True):
    """J^H applied to cotangents v (of g = H x^{m-1}) and phi (of f = H x^m).

    Returns (grad_x, grad_h)."""
    h, x = _c128(h), _c128(x)
    n = len(x)
    if len(h) != m * (n - 1) + 1:
        raise ValueError("h must have m(n-1)+1 entries")
    v = None if v is None else _c128(v)
    ph = None if phi is None else np.array([phi], np.complex128)
    gx = np.empty(n, np.complex128) if want_grad_x else None
    gh = np.empty(len(h), np.complex128) if want_grad_h else None
    _check(_lib().hko_tvp_backward(m, n, _ptr(h), _ptr(x), _ptr(v), _ptr(ph), _ptr(gx), _ptr(gh)),
           "tvp_backward")
    return gx, gh


def mode_backward(m: int, dims, h, vectors, v=None, phi=None, want=None, want_grad_h: bool = True):
    """J^H of y = H x_2 ... x_m (cotangent v) and alpha = H x_1 ... x_m (cotangent
    phi) with distinct vectors (hko_mode_backward).  vectors[0] is needed only
    with phi.  want[p] selects grad_{x_p} (default: all).  Returns
    (list of grad_{x_p} or None, grad_h or None)."""
    dims = np.ascontiguousarray(np.asarray(dims, np.int64))
    h = _c128(h)
    vecs = [None if a is None else _c128(a) for a in vectors]
    want = [True] * m if want is None else list(want)
    v = None if v is None else _c128(v)
    ph = None if phi is None else np.array([phi], np.complex128)
    gv = [np.empty(int(dims[p]), np.complex128) if want[p] else None for p in range(m)]
    gh = np.empty(len(h), np.complex128) if want_grad_h else None
    keep = _vec_ptrs(vecs)
    gkeep = _vec_ptrs(gv)
    _check(_lib().hko_mode_backward(m, _ptr(dims), _ptr(h), keep, _ptr(v), _ptr(ph), gkeep, _ptr(gh)),
           "mode_backward")
    return gv, gh


def block_backward(m: int, dims, block_dims, H, vectors, v=None, phi=None, want=None, want_grad_h: bool = True):
    """J^H of the BHHB product y = H x_2 ... x_m (vec(Y), cotangent v of n_1 N_1
    values) and alpha = H x_1 ... x_m (cotangent phi), distinct vectors
    (hko_block_backward).  Returns (list of grad vec(X_p) or None, grad vec(H) or None)."""
    dims = np.ascontiguousarray(np.asarray(dims, np.int64))
    bd = np.ascontiguousarray(np.asarray(block_dims, np.int64))
    H = _c128(H)
    vecs = [None if a is None else _c128(a) for a in vectors]
    want = [True] * m if want is None else list(want)
    v = None if v is None else _c128(v)
    ph = None if phi is None else np.array([phi], np.complex128)
    gv = [np.empty(int(dims[p] * bd[p]), np.complex128) if want[p] else None for p in range(m)]
    gh = np.empty(len(H), np.complex128) if want_grad_h else None
    keep = _vec_ptrs(vecs)
    gkeep = _vec_ptrs(gv)
    _check(_lib().hko_block_backward(m, _ptr(dims), _ptr(bd), _ptr(H), keep, _ptr(v), _ptr(ph), gkeep, _ptr(gh)),
           "block_backward")
    return gv, gh


def spectrum(a, N: int, idx=None, inverse: bool = False) -> np.ndarray:
    """Section 3 spectra as plain DFT sums (no FFT): fft(pad_N a) at the bins
    idx (all N bins when idx is None), or with inverse=True ifft(pad_N a)
    = (1/N) sum_s a_s e^{+2 pi i j s / N}, the h^ of the fast procedures."""
    a = _c128(a)
    idx = np.arange(N, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx), np.complex128)
    _check(_lib().hko_dft_sampled(1 if inverse else -1, _ptr(a), len(a), int(N), _ptr(idx), len(idx), _ptr(out)),
           "dft")
    return out


def tensor_matrix(m: int, h, U) -> np.ndarray:
    """Hankel tensor-matrix product T = H x_2 U x_3 U ... x_m U (Section 4.2) of the
    square order-m Hankel tensor (generating vector h, size n per mode) with the
    n x R matrix U in every mode but the first, with the Section 2.1 mode product
    (sum over i_p of H[.., i_p, ..] U[i_p, j_p]).

    Column (j_2, ..., j_m) of T is the tensor-vector product H x_2 U[:, j_2] ...
    x_m U[:, j_m] (the relation Section 4.2 states), evaluated by the direct oracle.
    Returns T as an n x R^(m-1) array whose column index is
    j_2 + R j_3 + ... + R^(m-2) j_m."""
    U = np.asarray(U, np.complex128)
    n, R = U.shape
    h = _c128(h)
    if len(h) != m * (n - 1) + 1:
        raise ValueError("h must have m(n-1)+1 entries")
    out = np.empty((n, R ** (m - 1)), np.complex128)
    for j in range(R ** (m - 1)):
        cols, r = [], j
        for _ in range(m - 1):
            cols.append(r % R)
            r //= R
        vecs = [None] + [U[:, c] for c in cols]
        out[:, j], _ = tvp(m, [n] * m, h, vecs)
    return out


def hankel_leading_subspace(h, rows: int, rank: int) -> np.ndarray:
    """R leading left singular vectors of the rows x (len(h) - rows + 1) Hankel
    matrix of h (the mode-1 unfolding of the Hankel tensor without its redundant
    columns, Section 4.2), by a dense SVD."""
    import scipy.linalg
    h = _c128(h)
    A = scipy.linalg.hankel(h[:rows], h[rows - 1:])
    Uf, _, _ = np.linalg.svd(A, full_matrices=False)
    return Uf[:, :rank]


def hooi(m: int, h, rank: int, iters: int, U0=None):
    """Algorithm 4.2 (HOOI for square Hankel tensors, U_1 = ... = U_m = U) in FP64
    with dense SVDs: U <- R leading left singular vectors of the Hankel matrix of
    h; then `iters` times U <- R leading left singular vectors of
    Unfold_1(H x_2 conj(U) ... x_m conj(U)); core S = H conj(U)^m.
    Returns (U, S) with S of shape (rank,)*m."""
    h = _c128(h)
    n = (len(h) + m - 1) // m
    U = hankel_leading_subspace(h, n, rank) if U0 is None else np.asarray(U0, np.complex128)
    for _ in range(iters):
        M = tensor_matrix(m, h, np.conj(U))
        Uf, _, _ = np.linalg.svd(M, full_matrices=False)
        U = Uf[:, :rank]
    M = tensor_matrix(m, h, np.conj(U))
    S = (np.conj(U).T @ M).reshape([rank] * m)   # axes (j_1, j_m, ..., j_2)
    S = np.transpose(S, [0] + list(range(m - 1, 0, -1)))
    return U, S


def problem_tvp(prob, want_y: Optional[bool] = None, want_alpha: Optional[bool] = None):
    """Oracle result for a ``workloads.Problem``."""
    wy = prob.want_y if want_y is None else want_y
    wa = prob.want_alpha if want_alpha is None else want_alpha
    if prob.is_block:
        return block_tvp(prob.m, prob.dims, prob.block_dims, prob.h, prob.vectors, wy, wa)
    return tvp(prob.m, prob.dims, prob.h, prob.vectors, wy, wa)
