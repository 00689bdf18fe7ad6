"""Python entry points with the names of the C ABI (marshalling only).

Every function takes torch tensors already resident on the GPU, allocates the
outputs and the workspace with torch (device memory and the current stream
are all torch provides here), and calls libhankel.so.  No arithmetic of the
product happens in Python.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import check, lib

_DT = {
    torch.complex64: _lib.HK_C64,
    torch.complex128: _lib.HK_C128,
    torch.float32: _lib.HK_F32,
    torch.float64: _lib.HK_F64,
}


def _dtype(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if t.is_conj() or t.is_neg():
        # a lazy conjugate / negative view: its memory holds the other values
        raise ValueError("tensor has a pending conjugation or negation; call .resolve_conj() / .resolve_neg()")
    return t


def _arg(t: torch.Tensor, name: str, numel: Optional[int] = None, dtype: Optional[torch.dtype] = None,
         device=None) -> torch.Tensor:
    """One tensor argument: on the GPU, contiguous, no pending conjugation, and
    (where given) the element count, dtype and device the call implies, so that
    no kernel reads or writes past the tensor's memory."""
    _dev(t)
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if numel is not None and t.numel() != int(numel):
        raise ValueError(f"{name} has {t.numel()} elements, expected {int(numel)}")
    return t


def _cotangent(t: Optional[torch.Tensor], name: str, numel: int, dtype: torch.dtype, device):
    """A cotangent handed over by autograd may be a lazy conjugate or negative
    view (its memory holds the other values): materialize it, then check it."""
    if t is None:
        return None
    t = t.resolve_conj().resolve_neg().contiguous()
    return _arg(t, name, numel, dtype, device)


def _spec_dtype(dtype: torch.dtype) -> torch.dtype:
    return {torch.float32: torch.complex64, torch.float64: torch.complex128}.get(dtype, dtype)


def _hlen(m: int, dims: Sequence[int]) -> int:
    return sum(int(d) for d in dims) - int(m) + 1


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> Tuple[Optional[torch.Tensor], int]:
    if nbytes == 0:
        return None, 0
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device), int(nbytes)


def _i64arr(vals):
    arr = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def _vecarr(vals):
    arr = (ctypes.c_void_p * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = None if v is None else v.data_ptr()
    return arr


def _same_device(*ts):
    devs = {t.device for t in ts if t is not None}
    if len(devs) > 1:
        raise ValueError("all tensors must be on one device")


def hankel_tvp(h: torch.Tensor, x: torch.Tensor, m: int, want_y: bool = True, want_alpha: bool = False):
    """Square Hankel tensor, equal vectors: (H x^{m-1}, H x^m).  Returns (y, alpha)."""
    _dev(x)
    n = x.numel()
    _arg(h, "h", m * (n - 1) + 1, x.dtype, x.device)
    dt = _dtype(x)
    y = torch.empty(n, dtype=x.dtype, device=x.device) if want_y else None
    alpha = torch.empty(1, dtype=x.dtype, device=x.device) if want_alpha else None
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_workspace_size(dt, m, n, ctypes.byref(nb)), "hankel_tvp_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().hankel_tvp(dt, _ptr(h), m, n, _ptr(x), _ptr(y), _ptr(alpha), _ptr(ws), wsb, _stream(x.device)),
          "hankel_tvp")
    return y, (None if alpha is None else alpha[0])


def hankel_tvp_noalloc(h: torch.Tensor, x: torch.Tensor, m: int, want_y: bool = True, want_alpha: bool = False):
    """hankel_tvp with the library's static device workspace (no workspace
    tensor is allocated; the outputs are the caller's only new tensors)."""
    _dev(x)
    n = x.numel()
    _arg(h, "h", m * (n - 1) + 1, x.dtype, x.device)
    dt = _dtype(x)
    y = torch.empty(n, dtype=x.dtype, device=x.device) if want_y else None
    alpha = torch.empty(1, dtype=x.dtype, device=x.device) if want_alpha else None
    check(lib().hankel_tvp_noalloc(dt, _ptr(h), m, n, _ptr(x), _ptr(y), _ptr(alpha), _stream(x.device)),
          "hankel_tvp_noalloc")
    return y, (None if alpha is None else alpha[0])


def hankel_mode_products(h: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], dims: Sequence[int] = None,
                         want_y: bool = True, want_alpha: bool = False):
    """General Hankel tensor: y = H x_2 ... x_m, alpha = H x_1 ... x_m.

    vectors[0] (x_1) may be None when want_alpha is False.  dims default to
    the vector lengths (dims[0] must be given if vectors[0] is None)."""
    m = len(vectors)
    if dims is None:
        if vectors[0] is None:
            raise ValueError("dims[0] is needed when vectors[0] is None")
        dims = [v.numel() for v in vectors]
    ref = next(v for v in vectors if v is not None)
    _dev(ref)
    if len(dims) != m:
        raise ValueError("dims must have one entry per vector")
    _arg(h, "h", _hlen(m, dims), ref.dtype, ref.device)
    for p, v in enumerate(vectors):
        if v is not None:
            _arg(v, f"vectors[{p}]", dims[p], ref.dtype, ref.device)
        elif p > 0 or want_alpha:
            raise ValueError(f"vectors[{p}] is needed")
    dt = _dtype(ref)
    y = torch.empty(int(dims[0]), dtype=ref.dtype, device=ref.device) if want_y else None
    alpha = torch.empty(1, dtype=ref.dtype, device=ref.device) if want_alpha else None
    d = _i64arr(dims)
    va = _vecarr(vectors)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_mode_products_workspace_size(dt, m, d, va, int(want_y), int(want_alpha), ctypes.byref(nb)),
          "hankel_mode_products_workspace_size")
    ws, wsb = _workspace(nb.value, ref.device)
    check(lib().hankel_mode_products(dt, _ptr(h), m, d, va, _ptr(y), _ptr(alpha), _ptr(ws), wsb,
                                     _stream(ref.device)), "hankel_mode_products")
    return y, (None if alpha is None else alpha[0])


def hankel_spectrum_layout(dtype: torch.dtype, m: int, dims: Sequence[int]) -> Tuple[int, int]:
    """(N, R) of the spectra of shape (m, dims): element r*R + c of a spectrum
    holds bin r + (N/R)*c of the length-N transform."""
    n_fft, row = ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib().hankel_spectrum_layout(_DT[dtype], m, _i64arr(dims), ctypes.byref(n_fft), ctypes.byref(row)),
          "hankel_spectrum_layout")
    return n_fft.value, row.value


def hankel_spectrum(src: torch.Tensor, m: int, dims: Sequence[int], which: int = -1) -> torch.Tensor:
    """Spectrum of h (which = -1: h^ = ifft(pad_N h)) or of the vector of mode
    `which` (x^ = fft(pad_N x)), in the library's row order (N elements)."""
    _dev(src)
    dt = _dtype(src)
    if len(dims) != m or not -1 <= which < m:
        raise ValueError("dims must have m entries and which must be in [-1, m)")
    _arg(src, "src", _hlen(m, dims) if which < 0 else dims[which])
    n_fft, _ = hankel_spectrum_layout(src.dtype, m, dims)
    cdt = _spec_dtype(src.dtype)
    spec = torch.empty(n_fft, dtype=cdt, device=src.device)
    d = _i64arr(dims)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_spectrum_workspace_size(dt, m, d, which, ctypes.byref(nb)), "hankel_spectrum_workspace_size")
    ws, wsb = _workspace(nb.value, src.device)
    check(lib().hankel_spectrum(dt, m, d, which, _ptr(src), _ptr(spec), _ptr(ws), wsb, _stream(src.device)),
          "hankel_spectrum")
    return spec


def hankel_mode_products_spectral(h_spec: torch.Tensor, m: int, dims: Sequence[int],
                                  vectors: Optional[Sequence[Optional[torch.Tensor]]] = None,
                                  specs: Optional[Sequence[Optional[torch.Tensor]]] = None,
                                  want_y: bool = True, want_alpha: bool = False,
                                  dtype: Optional[torch.dtype] = None):
    """Mode products from h^ (hankel_spectrum(h, m, dims)); mode p's operand is
    specs[p] (a spectrum) if given, else vectors[p].  dtype: the problem's
    dtype (default: that of the plain vectors, else the spectra's complex
    dtype); real problems return real y and alpha.  Returns (y, alpha)."""
    _dev(h_spec)
    if dtype is None:
        plain = [v for v in (vectors or []) if v is not None]
        dtype = plain[0].dtype if plain else h_spec.dtype
    dt = _DT[dtype]
    if len(dims) != m:
        raise ValueError("dims must have m entries")
    n_fft, _ = hankel_spectrum_layout(dtype, m, dims)
    sdt = _spec_dtype(dtype)
    _arg(h_spec, "h_spec", n_fft, sdt)
    for p in range(m):
        sp = specs[p] if specs is not None and p < len(specs) else None
        v = vectors[p] if vectors is not None and p < len(vectors) else None
        if sp is not None:
            _arg(sp, f"specs[{p}]", n_fft, sdt, h_spec.device)
        elif v is not None:
            _arg(v, f"vectors[{p}]", dims[p], dtype, h_spec.device)
        elif p > 0 or want_alpha:
            raise ValueError(f"mode {p} needs a vector or a spectrum")
    y = torch.empty(int(dims[0]), dtype=dtype, device=h_spec.device) if want_y else None
    alpha = torch.empty(1, dtype=dtype, device=h_spec.device) if want_alpha else None
    d = _i64arr(dims)
    va = _vecarr(list(vectors)) if vectors is not None else None
    sa = _vecarr(list(specs)) if specs is not None else None
    nb = ctypes.c_size_t(0)
    check(lib().hankel_mode_products_spectral_workspace_size(dt, m, d, va, sa, int(want_y), int(want_alpha),
                                                             ctypes.byref(nb)),
          "hankel_mode_products_spectral_workspace_size")
    ws, wsb = _workspace(nb.value, h_spec.device)
    check(lib().hankel_mode_products_spectral(dt, _ptr(h_spec), m, d, va, sa, _ptr(y), _ptr(alpha), _ptr(ws), wsb,
                                              _stream(h_spec.device)), "hankel_mode_products_spectral")
    return y, (None if alpha is None else alpha[0])


def hankel_tvp_spectral_strided_batched(h_spec: torch.Tensor, X: torch.Tensor, m: int, want_y: bool = True,
                                        want_alpha: bool = False):
    """Batch of equal-vector products H x_b^{m-1}, H x_b^m (X is (B, n)) sharing
    one stored h^ = hankel_spectrum(h, m, [n] * m).  Returns (Y (B, n), alpha (B))."""
    _dev(X)
    B, n = X.shape
    dt = _dtype(X)
    n_fft, _ = hankel_spectrum_layout(X.dtype, m, [n] * m)
    _arg(h_spec, "h_spec", n_fft, _spec_dtype(X.dtype), X.device)
    Y = torch.empty(B, n, dtype=X.dtype, device=X.device) if want_y else None
    alpha = torch.empty(B, dtype=X.dtype, device=X.device) if want_alpha else None
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_spectral_strided_batched_workspace_size(dt, m, n, B, ctypes.byref(nb)),
          "hankel_tvp_spectral_strided_batched_workspace_size")
    ws, wsb = _workspace(nb.value, X.device)
    check(lib().hankel_tvp_spectral_strided_batched(dt, _ptr(h_spec), m, n, _ptr(X), n, _ptr(Y), n, _ptr(alpha), B,
                                                    _ptr(ws), wsb, _stream(X.device)),
          "hankel_tvp_spectral_strided_batched")
    return Y, alpha


def block_hankel_tvp(H: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], inner_dims: Sequence[int],
                     block_dims: Sequence[int], want_y: bool = True, want_alpha: bool = False):
    """BHHB tensor: H is the column-major generating matrix (flat); vectors are vec(X_p)."""
    m = len(vectors)
    ref = next(v for v in vectors if v is not None)
    _dev(ref)
    if len(inner_dims) != m or len(block_dims) != m:
        raise ValueError("inner_dims and block_dims must have one entry per vector")
    _arg(H, "H", _hlen(m, inner_dims) * _hlen(m, block_dims), ref.dtype, ref.device)
    for p, v in enumerate(vectors):
        if v is not None:
            _arg(v, f"vectors[{p}]", int(inner_dims[p]) * int(block_dims[p]), ref.dtype, ref.device)
        elif p > 0 or want_alpha:
            raise ValueError(f"vectors[{p}] is needed")
    dt = _dtype(ref)
    ny = int(inner_dims[0]) * int(block_dims[0])
    y = torch.empty(ny, dtype=ref.dtype, device=ref.device) if want_y else None
    alpha = torch.empty(1, dtype=ref.dtype, device=ref.device) if want_alpha else None
    di, db = _i64arr(inner_dims), _i64arr(block_dims)
    va = _vecarr(vectors)
    nb = ctypes.c_size_t(0)
    check(lib().block_hankel_tvp_workspace_size(dt, m, di, db, va, int(want_y), int(want_alpha), ctypes.byref(nb)),
          "block_hankel_tvp_workspace_size")
    ws, wsb = _workspace(nb.value, ref.device)
    check(lib().block_hankel_tvp(dt, _ptr(H), m, di, db, va, _ptr(y), _ptr(alpha), _ptr(ws), wsb,
                                 _stream(ref.device)), "block_hankel_tvp")
    return y, (None if alpha is None else alpha[0])


def _adjoint_distinct(block: bool, h: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], inner_dims,
                      block_dims, grad_y, grad_alpha, want, want_grad_h: bool):
    m = len(vectors)
    ref = next(v for v in vectors if v is not None)
    _dev(ref)
    dt = _dtype(ref)
    if len(inner_dims) != m or (block and len(block_dims) != m):
        raise ValueError("dims must have one entry per vector")
    lens = [int(inner_dims[p]) * (int(block_dims[p]) if block else 1) for p in range(m)]
    hlen = _hlen(m, inner_dims) * (_hlen(m, block_dims) if block else 1)
    _arg(h, "H" if block else "h", hlen, ref.dtype, ref.device)
    for p, v in enumerate(vectors):
        if v is not None:
            _arg(v, f"vectors[{p}]", lens[p], ref.dtype, ref.device)
        elif p > 0 or grad_alpha is not None:
            raise ValueError(f"vectors[{p}] is needed")
    want = [True] * m if want is None else list(want)
    gy = _cotangent(grad_y, "grad_y", lens[0], ref.dtype, ref.device)
    ga = _cotangent(grad_alpha, "grad_alpha", 1, ref.dtype, ref.device)
    gv = [torch.empty(lens[p], dtype=ref.dtype, device=ref.device) if want[p] else None for p in range(m)]
    gh = torch.empty(hlen, dtype=ref.dtype, device=ref.device) if want_grad_h else None
    mask = sum(1 << p for p in range(m) if want[p])
    di = _i64arr(inner_dims)
    nb = ctypes.c_size_t(0)
    if block:
        db = _i64arr(block_dims)
        check(lib().block_hankel_tvp_backward_workspace_size(dt, m, di, db, mask, int(want_grad_h), ctypes.byref(nb)),
              "block_hankel_tvp_backward_workspace_size")
    else:
        check(lib().hankel_mode_products_backward_workspace_size(dt, m, di, mask, int(want_grad_h), ctypes.byref(nb)),
              "hankel_mode_products_backward_workspace_size")
    ws, wsb = _workspace(nb.value, ref.device)
    va, ga_arr = _vecarr(vectors), _vecarr(gv)
    if block:
        check(lib().block_hankel_tvp_backward(dt, _ptr(h), m, di, db, va, _ptr(gy), _ptr(ga), ga_arr, _ptr(gh),
                                              _ptr(ws), wsb, _stream(ref.device)), "block_hankel_tvp_backward")
    else:
        check(lib().hankel_mode_products_backward(dt, _ptr(h), m, di, va, _ptr(gy), _ptr(ga), ga_arr, _ptr(gh),
                                                  _ptr(ws), wsb, _stream(ref.device)), "hankel_mode_products_backward")
    return gv, gh


def hankel_mode_products_backward(h: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], dims: Sequence[int],
                                  grad_y: Optional[torch.Tensor], grad_alpha: Optional[torch.Tensor],
                                  want: Optional[Sequence[bool]] = None, want_grad_h: bool = True):
    """J^H of y = H x_2 ... x_m and alpha = H x_1 ... x_m (distinct vectors)
    applied to the cotangents grad_y (dims[0]) and grad_alpha (scalar).
    vectors[0] may be None when grad_alpha is None.  Returns (list of
    grad_{x_p} (None where want[p] is False), grad_h)."""
    return _adjoint_distinct(False, h, vectors, dims, None, grad_y, grad_alpha, want, want_grad_h)


def block_hankel_tvp_backward(H: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], inner_dims: Sequence[int],
                              block_dims: Sequence[int], grad_y: Optional[torch.Tensor],
                              grad_alpha: Optional[torch.Tensor], want: Optional[Sequence[bool]] = None,
                              want_grad_h: bool = True):
    """J^H of the BHHB products (vectors vec(X_p), y = vec(Y)) applied to
    grad_y (n_1 N_1) and grad_alpha.  Returns (list of grad vec(X_p), grad vec(H))."""
    return _adjoint_distinct(True, H, vectors, inner_dims, block_dims, grad_y, grad_alpha, want, want_grad_h)


def block_hankel_tvp_layout(dtype: torch.dtype, m: int, inner_dims: Sequence[int], block_dims: Sequence[int],
                            batch: int = 1) -> Tuple[int, int]:
    """(rows, cols) of the transform grid of a BHHB shape (each axis 2^k, 3 * 2^k or 5 * 2^k)."""
    r, c = ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib().block_hankel_tvp_layout(_DT[dtype], m, _i64arr(inner_dims), _i64arr(block_dims), int(batch),
                                        ctypes.byref(r), ctypes.byref(c)), "block_hankel_tvp_layout")
    return r.value, c.value


def block_hankel_tvp_levels(G: torch.Tensor, vectors: Sequence[Optional[torch.Tensor]], dims,
                            want_y: bool = True, want_alpha: bool = False):
    """Level-k block Hankel tensor (k = len(dims)): G is the column-major
    generating tensor (flat), dims[t][p] the size of mode p at level t
    (t = 0 innermost), vectors[p] = vec(X_p) column-major.  Returns (y, alpha)
    with y = vec(Y), Y of size dims[0][0] x dims[1][0] x ..."""
    m = len(vectors)
    k = len(dims)
    ref = next(v for v in vectors if v is not None)
    _dev(ref)
    if any(len(dims[t]) != m for t in range(k)):
        raise ValueError("dims[t] must have one entry per vector")
    glen = 1
    for t in range(k):
        glen *= _hlen(m, dims[t])
    _arg(G, "G", glen, ref.dtype, ref.device)
    for p, v in enumerate(vectors):
        if v is not None:
            vlen = 1
            for t in range(k):
                vlen *= int(dims[t][p])
            _arg(v, f"vectors[{p}]", vlen, ref.dtype, ref.device)
        elif p > 0 or want_alpha:
            raise ValueError(f"vectors[{p}] is needed")
    dt = _dtype(ref)
    flat = [int(dims[t][p]) for t in range(k) for p in range(m)]
    ny = 1
    for t in range(k):
        ny *= int(dims[t][0])
    y = torch.empty(ny, dtype=ref.dtype, device=ref.device) if want_y else None
    alpha = torch.empty(1, dtype=ref.dtype, device=ref.device) if want_alpha else None
    da = _i64arr(flat)
    va = _vecarr(vectors)
    nb = ctypes.c_size_t(0)
    check(lib().block_hankel_tvp_levels_workspace_size(dt, m, k, da, va, int(want_y), int(want_alpha),
                                                       ctypes.byref(nb)), "block_hankel_tvp_levels_workspace_size")
    ws, wsb = _workspace(nb.value, ref.device)
    check(lib().block_hankel_tvp_levels(dt, _ptr(G), m, k, da, va, _ptr(y), _ptr(alpha), _ptr(ws), wsb,
                                        _stream(ref.device)), "block_hankel_tvp_levels")
    return y, (None if alpha is None else alpha[0])


def hankel_tvp_backward(h: torch.Tensor, x: torch.Tensor, m: int, grad_y: Optional[torch.Tensor],
                        grad_alpha: Optional[torch.Tensor], want_grad_x: bool = True, want_grad_h: bool = True):
    """J^H [grad_y; grad_alpha] for g = H x^{m-1}, f = H x^m.  Returns (grad_x, grad_h)."""
    _dev(x)
    n = x.numel()
    dt = _dtype(x)
    _arg(h, "h", m * (n - 1) + 1, x.dtype, x.device)
    gx = torch.empty(n, dtype=x.dtype, device=x.device) if want_grad_x else None
    gh = torch.empty(h.numel(), dtype=x.dtype, device=x.device) if want_grad_h else None
    ga = _cotangent(grad_alpha, "grad_alpha", 1, x.dtype, x.device)
    gy = _cotangent(grad_y, "grad_y", n, x.dtype, x.device)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_backward_workspace_size(dt, m, n, ctypes.byref(nb)), "hankel_tvp_backward_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().hankel_tvp_backward(dt, _ptr(h), m, n, _ptr(x), _ptr(gy), _ptr(ga), _ptr(gx), _ptr(gh), _ptr(ws), wsb,
                                    _stream(x.device)), "hankel_tvp_backward")
    return gx, gh


def hankel_tvp_backward_spectral(h: torch.Tensor, x_spec: torch.Tensor, m: int, n: int,
                                 grad_y: Optional[torch.Tensor], grad_alpha: Optional[torch.Tensor],
                                 want_grad_x: bool = True, want_grad_h: bool = True):
    """hankel_tvp_backward with x given by its stored spectrum
    (hankel_spectrum(x, m, [n] * m, 1)).  Returns (grad_x, grad_h)."""
    _dev(h)
    dt = _dtype(h)
    _arg(h, "h", m * (n - 1) + 1)
    n_fft, _ = hankel_spectrum_layout(h.dtype, m, [n] * m)
    _arg(x_spec, "x_spec", n_fft, _spec_dtype(h.dtype), h.device)
    gx = torch.empty(n, dtype=h.dtype, device=h.device) if want_grad_x else None
    gh = torch.empty(h.numel(), dtype=h.dtype, device=h.device) if want_grad_h else None
    ga = _cotangent(grad_alpha, "grad_alpha", 1, h.dtype, h.device)
    gy = _cotangent(grad_y, "grad_y", n, h.dtype, h.device)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_backward_spectral_workspace_size(dt, m, n, ctypes.byref(nb)),
          "hankel_tvp_backward_spectral_workspace_size")
    ws, wsb = _workspace(nb.value, h.device)
    check(lib().hankel_tvp_backward_spectral(dt, _ptr(h), m, n, _ptr(x_spec), _ptr(gy), _ptr(ga), _ptr(gx), _ptr(gh),
                                             _ptr(ws), wsb, _stream(h.device)), "hankel_tvp_backward_spectral")
    return gx, gh


def hankel_tvp_save_spectrum(h: torch.Tensor, x: torch.Tensor, m: int, want_y: bool = True,
                             want_alpha: bool = False):
    """Equal-vector products that also return x^ for the adjoint: h (d_H) and x
    (n) for one product, or h (B, d_H) and x (B, n) for a batch.  Returns
    (y, alpha, x_spec) with x_spec (N) or (B, N) in the row order of
    hankel_spectrum."""
    _dev(x)
    single = x.dim() == 1
    X = x.reshape(1, -1) if single else x
    B, n = X.shape
    dt = _dtype(x)
    d_h = m * (n - 1) + 1
    _arg(h, "h", B * d_h, x.dtype, x.device)
    if not single and h.dim() != 2:
        raise ValueError("h must be (B, d_H)")
    n_fft, _ = hankel_spectrum_layout(x.dtype, m, [n] * m)
    y = torch.empty(B, n, dtype=x.dtype, device=x.device) if want_y else None
    alpha = torch.empty(B, dtype=x.dtype, device=x.device) if want_alpha else None
    spec = torch.empty(B, n_fft, dtype=_spec_dtype(x.dtype), device=x.device)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_save_spectrum_workspace_size(dt, m, n, B, ctypes.byref(nb)),
          "hankel_tvp_save_spectrum_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().hankel_tvp_save_spectrum(dt, _ptr(h), d_h, m, n, _ptr(X), n, _ptr(y), n, _ptr(alpha), _ptr(spec),
                                         n_fft, B, _ptr(ws), wsb, _stream(x.device)), "hankel_tvp_save_spectrum")
    if single:
        return (None if y is None else y[0]), (None if alpha is None else alpha[0]), spec[0]
    return y, alpha, spec


def hankel_tvp_backward_spectral_strided_batched(h: torch.Tensor, x_spec: torch.Tensor, m: int, n: int,
                                                 grad_y: Optional[torch.Tensor], grad_alpha: Optional[torch.Tensor],
                                                 want_grad_x: bool = True, want_grad_h: bool = True):
    """J^H of a strided batch with x given by its stored spectra: h (B, d_H),
    x_spec (B, N) from hankel_tvp_save_spectrum, grad_y (B, n), grad_alpha (B,).
    Returns (grad_x (B, n), grad_h (B, d_H))."""
    _dev(h)
    if h.dim() != 2:
        raise ValueError("h must be (B, d_H)")
    B = h.shape[0]
    dt = _dtype(h)
    d_h = m * (n - 1) + 1
    _arg(h, "h", B * d_h)
    n_fft, _ = hankel_spectrum_layout(h.dtype, m, [n] * m)
    _arg(x_spec, "x_spec", B * n_fft, _spec_dtype(h.dtype), h.device)
    gx = torch.empty(B, n, dtype=h.dtype, device=h.device) if want_grad_x else None
    gh = torch.empty(B, d_h, dtype=h.dtype, device=h.device) if want_grad_h else None
    ga = _cotangent(grad_alpha, "grad_alpha", B, h.dtype, h.device)
    gy = _cotangent(grad_y, "grad_y", B * n, h.dtype, h.device)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_backward_spectral_strided_batched_workspace_size(dt, m, n, B, ctypes.byref(nb)),
          "hankel_tvp_backward_spectral_strided_batched_workspace_size")
    ws, wsb = _workspace(nb.value, h.device)
    check(lib().hankel_tvp_backward_spectral_strided_batched(dt, _ptr(h), d_h, m, n, _ptr(x_spec), n_fft, _ptr(gy), n,
                                                             _ptr(ga), _ptr(gx), n, _ptr(gh), d_h, B, _ptr(ws), wsb,
                                                             _stream(h.device)),
          "hankel_tvp_backward_spectral_strided_batched")
    return gx, gh


def hankel_tvp_strided_batched(h: torch.Tensor, x: torch.Tensor, m: int, want_y: bool = True,
                               want_alpha: bool = False):
    """Batch of equal-vector products: h (B, d_H), x (B, n).  Returns (y (B, n), alpha (B,))."""
    _dev(x)
    B, n = x.shape
    dt = _dtype(x)
    _arg(h, "h", B * (m * (n - 1) + 1), x.dtype, x.device)
    if h.dim() != 2:
        raise ValueError("h must be (B, d_H)")
    y = torch.empty(B, n, dtype=x.dtype, device=x.device) if want_y else None
    alpha = torch.empty(B, dtype=x.dtype, device=x.device) if want_alpha else None
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_strided_batched_workspace_size(dt, m, n, B, ctypes.byref(nb)),
          "hankel_tvp_strided_batched_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().hankel_tvp_strided_batched(dt, _ptr(h), h.shape[1], m, n, _ptr(x), n, _ptr(y), n, _ptr(alpha), B,
                                           _ptr(ws), wsb, _stream(x.device)), "hankel_tvp_strided_batched")
    return y, alpha


def hankel_tvp_backward_strided_batched(h: torch.Tensor, x: torch.Tensor, m: int, grad_y: Optional[torch.Tensor],
                                        grad_alpha: Optional[torch.Tensor], want_grad_x: bool = True,
                                        want_grad_h: bool = True):
    """J^H of a strided batch: h (B, d_H), x (B, n), grad_y (B, n), grad_alpha (B,).
    Returns (grad_x (B, n), grad_h (B, d_H))."""
    _dev(x)
    B, n = x.shape
    dt = _dtype(x)
    _arg(h, "h", B * (m * (n - 1) + 1), x.dtype, x.device)
    if h.dim() != 2:
        raise ValueError("h must be (B, d_H)")
    gx = torch.empty(B, n, dtype=x.dtype, device=x.device) if want_grad_x else None
    gh = torch.empty(B, h.shape[1], dtype=x.dtype, device=x.device) if want_grad_h else None
    gy = _cotangent(grad_y, "grad_y", B * n, x.dtype, x.device)
    ga = _cotangent(grad_alpha, "grad_alpha", B, x.dtype, x.device)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tvp_backward_strided_batched_workspace_size(dt, m, n, B, ctypes.byref(nb)),
          "hankel_tvp_backward_strided_batched_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().hankel_tvp_backward_strided_batched(
        dt, _ptr(h), h.shape[1], m, n, _ptr(x), n, _ptr(gy), n, _ptr(ga), _ptr(gx), n, _ptr(gh), h.shape[1], B,
        _ptr(ws), wsb, _stream(x.device)), "hankel_tvp_backward_strided_batched")
    return gx, gh


def block_hankel_tvp_strided_batched(H: torch.Tensor, x: torch.Tensor, m: int, inner: int, blocks: int,
                                     want_y: bool = True, want_alpha: bool = False):
    """Batch of equal-vector BHHB products: H (B, rows*cols) column-major, x (B, inner*blocks)."""
    _dev(x)
    B = x.shape[0]
    dt = _dtype(x)
    if x.dim() != 2 or x.shape[1] != inner * blocks:
        raise ValueError("x must be (B, inner * blocks)")
    _arg(H, "H", B * (m * (inner - 1) + 1) * (m * (blocks - 1) + 1), x.dtype, x.device)
    if H.dim() != 2:
        raise ValueError("H must be (B, rows * cols)")
    ny = inner * blocks
    y = torch.empty(B, ny, dtype=x.dtype, device=x.device) if want_y else None
    alpha = torch.empty(B, dtype=x.dtype, device=x.device) if want_alpha else None
    di, db = _i64arr([inner] * m), _i64arr([blocks] * m)
    nb = ctypes.c_size_t(0)
    check(lib().block_hankel_tvp_strided_batched_workspace_size(dt, m, di, db, B, ctypes.byref(nb)),
          "block_hankel_tvp_strided_batched_workspace_size")
    ws, wsb = _workspace(nb.value, x.device)
    check(lib().block_hankel_tvp_strided_batched(dt, _ptr(H), H.shape[1], m, di, db, _ptr(x), x.shape[1], _ptr(y), ny,
                                                 _ptr(alpha), B, _ptr(ws), wsb, _stream(x.device)),
          "block_hankel_tvp_strided_batched")
    return y, alpha


def _problem_array(problems):
    """hk_problem_t array of a sequence of problem dicts (keys m, dims, h,
    vectors, optional block_dims, want_y, want_alpha), with the outputs it
    allocates.  Returns (array, [(y, alpha)], tensors to keep alive, dtype,
    device)."""
    arr = (_lib.hk_problem_t * max(1, len(problems)))()
    dtype = None
    keep, outputs = [], []
    ref = None
    for i, p in enumerate(problems):
        vecs = p["vectors"]
        ref = next((v for v in vecs if v is not None), None)
        if ref is None:
            raise ValueError(f"problem {i}: no vector given")
        _dev(ref)
        dtype = ref.dtype if dtype is None else dtype
        if ref.dtype != dtype:
            raise TypeError("all problems of a batch share one dtype")
        m = p["m"]
        dims = p["dims"]
        bd = p.get("block_dims")
        want_y = p.get("want_y", True)
        want_a = p.get("want_alpha", False)
        if len(vecs) != m or len(dims) != m or (bd is not None and len(bd) != m):
            raise ValueError(f"problem {i}: vectors, dims and block_dims need m entries")
        hlen = _hlen(m, dims) * (_hlen(m, bd) if bd is not None else 1)
        _arg(p["h"], f"problem {i} h", hlen, dtype, ref.device)
        for k, v in enumerate(vecs):
            if v is not None:
                _arg(v, f"problem {i} vectors[{k}]", int(dims[k]) * (int(bd[k]) if bd is not None else 1),
                     dtype, ref.device)
            elif k > 0 or want_a:
                raise ValueError(f"problem {i}: vectors[{k}] is needed")
        ny = int(dims[0]) * (int(bd[0]) if bd is not None else 1)
        y = torch.empty(ny, dtype=dtype, device=ref.device) if want_y else None
        a = torch.empty(1, dtype=dtype, device=ref.device) if want_a else None
        outputs.append((y, a))
        keep.extend([y, a, p["h"]] + list(vecs))
        q = arr[i]
        q.m = m
        q.is_block = 1 if bd is not None else 0
        for k in range(m):
            q.dims[k] = int(dims[k])
            q.block_dims[k] = int(bd[k]) if bd is not None else 0
            q.vectors[k] = None if vecs[k] is None else vecs[k].data_ptr()
        q.h = p["h"].data_ptr()
        q.y = None if y is None else y.data_ptr()
        q.alpha = None if a is None else a.data_ptr()
    device = ref.device if ref is not None else torch.device("cuda")
    return arr, outputs, keep, dtype, device


def _batched_oneshot(name: str, problems):
    arr, outputs, keep, dtype, device = _problem_array(list(problems))
    if not problems:
        return outputs
    dt = _DT[dtype]
    nb = ctypes.c_size_t(0)
    check(getattr(lib(), name + "_workspace_size")(dt, arr, len(problems), ctypes.byref(nb)),
          name + "_workspace_size")
    ws, ws_bytes = _workspace(max(256, nb.value), device)
    check(getattr(lib(), name)(dt, arr, len(problems), _ptr(ws), ws_bytes, _stream(device)), name)
    return outputs


def hankel_mode_products_batched(problems):
    """One-shot batch of general (1D) Hankel products through the C entry
    point hankel_mode_products_batched; every problem without block_dims.
    Returns a list of (y, alpha) per problem."""
    return _batched_oneshot("hankel_mode_products_batched", problems)


def block_hankel_tvp_batched(problems):
    """One-shot batch of BHHB products (every problem with block_dims) through
    the C entry point block_hankel_tvp_batched.  Returns a list of (y, alpha)."""
    return _batched_oneshot("block_hankel_tvp_batched", problems)


class Plan:
    """A batched plan over heterogeneous problems (hk_plan_*).

    problems: sequence of dicts with keys m, dims, h, vectors, and optionally
    block_dims (BHHB), want_y (default True), want_alpha (default False).
    The plan allocates each problem's outputs; results are in .outputs."""

    def __init__(self, problems, flags: int = 0):
        self.problems = list(problems)
        arr, self.outputs, self._keep, dtype, self.device = _problem_array(self.problems)
        self.dt = _DT[dtype] if dtype is not None else _lib.HK_C64
        self._arr = arr
        self._plan = ctypes.c_void_p()
        check(lib().hk_plan_create(ctypes.byref(self._plan), self.dt, arr, len(self.problems), flags),
              "hk_plan_create")
        nb = ctypes.c_size_t(0)
        check(lib().hk_plan_workspace_size(self._plan, ctypes.byref(nb)), "hk_plan_workspace_size")
        self.ws, self.ws_bytes = _workspace(max(256, nb.value), self.device)

    def execute(self):
        check(lib().hk_plan_execute(self._plan, _ptr(self.ws), self.ws_bytes, _stream(self.device)), "hk_plan_execute")
        return self.outputs

    def status(self):
        check(lib().hk_plan_status(self._plan), "hk_plan_status")

    def pass_bytes(self) -> int:
        """Bytes one execute reads and writes under the pass model of its kernels."""
        b = ctypes.c_int64(0)
        check(lib().hk_plan_pass_bytes(self._plan, ctypes.byref(b)), "hk_plan_pass_bytes")
        return int(b.value)

    def tune_times(self):
        """HK_PLAN_AUTOTUNE: (ms per execute of the default plan, of the kept plan,
        mask of length buckets moved to powers of two); zeros before the first execute."""
        a, b, mask = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_uint32(0)
        check(lib().hk_plan_tune_times(self._plan, ctypes.byref(a), ctypes.byref(b), ctypes.byref(mask)),
              "hk_plan_tune_times")
        return a.value, b.value, int(mask.value)

    def set_wait_bound(self, spins: int):
        """Persistent plans: barrier polling iterations before the error path (diagnostics)."""
        check(lib().hk_plan_set_wait_bound(self._plan, int(spins)), "hk_plan_set_wait_bound")

    def close(self):
        if self._plan:
            lib().hk_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hankel_tensor_matrix(h: torch.Tensor, U: torch.Tensor, m: int) -> torch.Tensor:
    """T = H x_2 U ... x_m U for the square order-m Hankel tensor with generating
    vector h and an (n, R) matrix U.  Returns T with shape (n, R, ..., R),
    T[i, j_2, ..., j_m] = (H x_2 U[:, j_2] ... x_m U[:, j_m])[i]."""
    if U.dim() != 2 or U.dtype != h.dtype or U.device != h.device:
        raise ValueError("U must be an (n, R) matrix of h's dtype on h's device")
    n, R = U.shape
    _arg(h, "h", m * (n - 1) + 1)
    if not U.is_cuda:
        raise ValueError("tensors must live on the GPU")
    dt = _dtype(h)
    Ucm = U.t().resolve_conj().resolve_neg().contiguous()  # column-major n x R: column j contiguous
    ncols = R ** (m - 1)
    out = torch.empty((ncols, n), dtype=h.dtype, device=h.device)  # column-major n x R^(m-1)
    nb = ctypes.c_size_t(0)
    check(lib().hankel_tensor_matrix_workspace_size(dt, m, n, R, ctypes.byref(nb)),
          "hankel_tensor_matrix_workspace_size")
    ws, wsb = _workspace(nb.value, h.device)
    check(lib().hankel_tensor_matrix(dt, _ptr(h), m, n, R, _ptr(Ucm), _ptr(out), _ptr(ws), wsb, _stream(h.device)),
          "hankel_tensor_matrix")
    # out rows are columns j = j_2 + R j_3 + ...: as a row-major array its axes are (j_m, ..., j_2, i)
    T = out.reshape([R] * (m - 1) + [n])
    return T.permute([m - 1] + list(range(m - 2, -1, -1)))


def hankel_tvp_batched(problems):
    """One-shot heterogeneous batch.  Returns a list of (y, alpha) per problem."""
    plan = Plan(problems)
    try:
        out = plan.execute()
        plan.status()
    finally:
        plan.close()
    return out


_LENGTHS = {"auto": 0, "pow2": 1, "smallest": 2}


def hk_set_fft_lengths(policy: str):
    """Process-wide transform lengths for later calls and plans: "auto"
    (default: the smallest of 2^k, 3 * 2^k, 5 * 2^k when instances * the
    power-of-two length >= 2^18, else the power of two), "smallest" or
    "pow2"."""
    if policy not in _LENGTHS:
        raise ValueError("policy must be 'auto', 'smallest' or 'pow2'")
    check(lib().hk_set_fft_lengths(_LENGTHS[policy]), "hk_set_fft_lengths")


def hk_get_fft_lengths() -> str:
    return {v: k for k, v in _LENGTHS.items()}[lib().hk_get_fft_lengths()]


def hk_fft_layout(d_h: int):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().hk_fft_layout(d_h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "hk_fft_layout")
    return a.value, b.value, c.value


def hk_autotune_tvp(dtype: torch.dtype, m: int, n: int, verbose: bool = False):
    check(lib().hk_autotune_tvp(_DT[dtype], m, n, int(verbose)), "hk_autotune_tvp")


def hk_autotune(dtype: torch.dtype, kind: str, m: int, n: int = 0, inner=None, blocks=None, batch: int = 1,
                verbose: bool = False):
    """kind: 'forward', 'adjoint' (1D equal-vector shapes) or 'block' (BHHB, inner/blocks per mode)."""
    k = {"forward": 0, "adjoint": 1, "block": 2}[kind]
    di = _i64arr(inner) if inner is not None else None
    db = _i64arr(blocks) if blocks is not None else None
    check(lib().hk_autotune(_DT[dtype], k, m, n, di, db, batch, int(verbose)), "hk_autotune")


def hk_tune_save(path: str):
    check(lib().hk_tune_save(str(path).encode()), "hk_tune_save")


def hk_tune_load(path: str) -> int:
    n = ctypes.c_int(0)
    check(lib().hk_tune_load(str(path).encode(), ctypes.byref(n)), "hk_tune_load")
    return n.value


def hk_last_launch_count() -> int:
    return int(lib().hk_last_launch_count())


PROF_KINDS = ("resident", "pass_a", "pass_b", "pass_d", "batch")


def hk_profile_start():
    check(lib().hk_profile_start(), "hk_profile_start")


def hk_profile_stop():
    """Returns {kind: (total_ms, launches)} for the kernels enqueued since start."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int64 * 5)()
    check(lib().hk_profile_stop(ms, cnt), "hk_profile_stop")
    return {PROF_KINDS[k]: (ms[k], cnt[k]) for k in range(5)}
