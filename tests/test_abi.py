"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/hankel.h, and rejects bad arguments on the host with the
documented status codes before anything is enqueued."""
import ctypes
import os

import pytest

from paper_1401_6238_amd import _lib

HK_C64, HK_C128, HK_F32, HK_F64 = 0, 1, 2, 3
OK, INVALID, NULLP, MISALIGNED, WORKSPACE, SIZE, DEVICE, HIP, FAULT, NOTSUP = range(10)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1401_6238_amd import build
        build.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _lib.header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), f"{n} declared in hankel.h but not exported"


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libhankel.so")
    with pytest.raises(ImportError):
        _lib.lib()


def ws(L, dt, m, n):
    b = ctypes.c_size_t(0)
    rc = L.hankel_tvp_workspace_size(dt, m, n, ctypes.byref(b))
    return rc, b.value


def test_workspace_sizes(L):
    assert ws(L, HK_C64, 3, 64) == (OK, 0)          # resident: no workspace
    rc, b = ws(L, HK_C64, 4, 1 << 18)               # N = 2^20, two buffers
    assert rc == OK and b == ((2 * (1 << 20) * 8 + 4096 * 8 + 255) // 256) * 256
    rc, b3 = ws(L, HK_C64, 3, 65536)                # d_H = 196606 -> N = 3 * 2^16
    assert rc == OK and b3 == ((2 * 3 * (1 << 16) * 8 + 4096 * 8 + 255) // 256) * 256
    rc, b128 = ws(L, HK_C128, 4, 1 << 18)
    assert rc == OK and b128 > b


@pytest.mark.parametrize("dt,m,n,code", [
    (7, 3, 10, INVALID), (HK_C64, 1, 10, INVALID), (HK_C64, 9, 10, INVALID), (HK_C64, 3, 0, INVALID),
    (HK_C64, 3, -5, INVALID), (HK_C64, 4, (1 << 23), SIZE), (HK_C128, 2, (1 << 24) + 1, SIZE),
])
def test_workspace_size_rejects(L, dt, m, n, code):
    assert ws(L, dt, m, n)[0] == code
    assert L.hk_last_error()


def test_null_bytes_pointer(L):
    assert L.hankel_tvp_workspace_size(HK_C64, 3, 10, None) == NULLP


def P(v):
    return ctypes.c_void_p(v)


def test_tvp_argument_errors_without_device(L):
    h, x, y = P(0x10000), P(0x20000), P(0x30000)
    assert L.hankel_tvp(HK_C64, h, 3, 10, x, None, None, None, 0, None) == NULLP       # no output
    assert L.hankel_tvp(HK_C64, None, 3, 10, x, y, None, None, 0, None) == NULLP       # no h
    assert L.hankel_tvp(HK_C64, P(0x10004), 3, 10, x, y, None, None, 0, None) == MISALIGNED
    assert L.hankel_tvp(HK_C128, h, 3, 10, P(0x20008), y, None, None, 0, None) == MISALIGNED
    # 3-pass size with no workspace
    assert L.hankel_tvp(HK_C64, h, 4, 1 << 18, x, y, None, None, 0, None) == WORKSPACE
    assert L.hankel_tvp(HK_C64, h, 4, 1 << 18, x, y, None, P(0x40000), 1024, None) == WORKSPACE
    assert b"workspace" in L.hk_last_error()


def test_mode_products_argument_errors(L):
    dims = (ctypes.c_int64 * 3)(5, 6, 7)
    vecs = (ctypes.c_void_p * 3)(0x1000, 0x2000, None)
    h, y = P(0x10000), P(0x30000)
    assert L.hankel_mode_products(HK_C64, h, 3, dims, vecs, y, None, None, 0, None) == NULLP  # x_3 missing
    vecs2 = (ctypes.c_void_p * 3)(None, 0x2000, 0x3000)
    assert L.hankel_mode_products(HK_C64, h, 3, dims, vecs2, None, P(0x5000), None, 0, None) == NULLP  # alpha needs x_1
    bad = (ctypes.c_int64 * 3)(5, 0, 7)
    assert L.hankel_mode_products(HK_C64, h, 3, bad, vecs2, y, None, None, 0, None) == INVALID
    assert L.hankel_mode_products(HK_C64, h, 3, None, vecs2, y, None, None, 0, None) == NULLP


def test_block_argument_errors(L):
    inner = (ctypes.c_int64 * 2)(3000, 2000)
    blocks = (ctypes.c_int64 * 2)(4, 4)
    vecs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    b = ctypes.c_size_t(0)
    # the padded grid would exceed 4096 rows
    assert L.block_hankel_tvp_workspace_size(HK_C64, 2, inner, blocks, vecs, 1, 0, ctypes.byref(b)) == SIZE
    inner = (ctypes.c_int64 * 2)(30, 20)
    assert L.block_hankel_tvp_workspace_size(HK_C64, 2, inner, blocks, vecs, 1, 0, ctypes.byref(b)) == OK
    assert b.value > 0


def test_backward_argument_errors(L):
    h, x, g = P(0x10000), P(0x20000), P(0x30000)
    assert L.hankel_tvp_backward(HK_F64, h, 3, 10, x, g, None, g, None, None, 0, None) == NOTSUP
    assert L.hankel_tvp_backward(HK_C64, h, 3, 10, x, g, None, None, None, None, 0, None) == NULLP


def test_plan_argument_errors(L):
    plan = ctypes.c_void_p()
    assert L.hk_plan_create(ctypes.byref(plan), HK_C64, None, 1, 1) == NULLP
    assert L.hk_plan_create(ctypes.byref(plan), HK_C64, None, -1, 1) == INVALID
    assert L.hk_plan_create(ctypes.byref(plan), HK_C64, None, 0, 0x100) == INVALID
    assert L.hk_plan_create(ctypes.byref(plan), HK_C64, None, 0, 0x3) == INVALID  # persistent + per-pass
    assert L.hk_plan_create(None, HK_C64, None, 0, 1) == NULLP


def fft_layout(L, d):
    a, r, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.hk_fft_layout(d, ctypes.byref(a), ctypes.byref(r), ctypes.byref(c)) == OK
    return a.value, r.value, c.value


def smooth_lengths(d):
    """Every length 2^k, 3 * 2^k, 5 * 2^k that is >= d (brute force)."""
    out = []
    for odd in (1, 3, 5):
        k = 0
        while odd << k < d:
            k += 1
        out.append(odd << k)
    return out


@pytest.fixture
def smallest(L):
    """Transform lengths: always the smallest with kernels (restored to auto)."""
    assert L.hk_set_fft_lengths(2) == OK
    yield
    assert L.hk_set_fft_lengths(0) == OK


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 190, 193, 1100, 1537, 4097, 5000, 6145, 12000, 40961,
                               196606, 786433, 1048573, (1 << 24) - 5])
def test_fft_layout(L, smallest, d):
    n, r, c = fft_layout(L, d)
    assert n >= d and n == min(smooth_lengths(d))    # the smallest 2^k, 3 * 2^k, 5 * 2^k >= d_H
    assert n % (r * c) == 0 and n // (r * c) in (1, 3, 5)
    assert r & (r - 1) == 0 and c & (c - 1) == 0


def test_fft_layout_cases(L, smallest):
    assert fft_layout(L, 1048573)[0] == 1 << 20       # the large single product stays a power of two
    assert fft_layout(L, 190) == (192, 64, 1)        # 3 sequences of 64, one workgroup holds it
    assert fft_layout(L, 1100) == (1280, 256, 1)     # 5 sequences of 256
    n, r, c = fft_layout(L, 12000)                   # 3 * 4096: multipass sequences
    assert n == 12288 and r * c == 4096 and c > 1
    a, r_, c_ = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.hk_fft_layout(0, ctypes.byref(a), ctypes.byref(r_), ctypes.byref(c_)) == INVALID


def test_status_strings(L):
    for code in range(10):
        assert L.hk_status_string(code)
    assert L.hk_version() > 0


def test_autotune_argument_errors(L):
    """Rejected before any device work: unknown kind, bad order, missing block dims."""
    assert L.hk_autotune(HK_C64, 7, 3, 64, None, None, 1, 0) == INVALID
    assert L.hk_autotune(HK_C64, 0, 1, 64, None, None, 1, 0) == INVALID
    assert L.hk_autotune(HK_C64, 2, 3, 0, None, None, 1, 0) == NULLP
    assert L.hk_autotune(HK_F32, 1, 3, 64, None, None, 1, 0) == NOTSUP
    assert L.hk_autotune_tvp(HK_C64, 3, 1 << 26, 0) == SIZE


def test_tune_db_round_trip(L, tmp_path):
    """The schedule database loads, merges and saves on the host."""
    good = tmp_path / "db.txt"
    good.write_text("# comment\n0 0 0 23 -1 0 : 8 1 16 8 0\n1 1 0 23 -1 2 : 16 2 8 4 -1 1\n")
    n = ctypes.c_int(-1)
    assert L.hk_tune_load(str(good).encode(), ctypes.byref(n)) == OK
    assert n.value == 2
    out = tmp_path / "out.txt"
    assert L.hk_tune_save(str(out).encode()) == OK
    lines = [ln for ln in out.read_text().splitlines() if not ln.startswith("#")]
    # lines without the odd factor are power-of-two lengths (odd = 1)
    assert "1 1 0 1 23 -1 2 : 16 2 8 4 -1 1 1" in lines
    assert "0 0 0 1 23 -1 0 : 8 1 16 8 0 0 1" in lines
    seven = tmp_path / "seven.txt"
    seven.write_text("0 0 0 22 -1 0 : 8 2 16 8 0 1 4\n0 0 0 3 16 -1 0 : 4 1 16 8 0 1 2\n")
    assert L.hk_tune_load(str(seven).encode(), None) == OK
    assert L.hk_tune_save(str(out).encode()) == OK
    assert "0 0 0 1 22 -1 0 : 8 2 16 8 0 1 4" in out.read_text()
    assert "0 0 0 3 16 -1 0 : 4 1 16 8 0 1 2" in out.read_text()
    bad_odd = tmp_path / "odd.txt"
    bad_odd.write_text("0 0 0 7 16 -1 0 : 4 1 16 8 0 1 2\n")  # no factor-7 kernels
    assert L.hk_tune_load(str(bad_odd).encode(), None) == INVALID
    three = tmp_path / "three.txt"
    three.write_text("0 0 0 20 -1 0 : 8 1 16 8 0 0 3\n")  # 3 rows in turn is not offered
    assert L.hk_tune_load(str(three).encode(), None) == INVALID
    three.write_text("0 0 0 20 -1 0 : 8 1 16 3 0 0 1\n")  # column tiles are powers of two wide
    assert L.hk_tune_load(str(three).encode(), None) == INVALID
    three.write_text("0 0 0 21 -1 0 : 8 3 16 4 0 0 1\n")  # any number of rows per workgroup
    assert L.hk_tune_load(str(three).encode(), None) == OK
    bad = tmp_path / "bad.txt"
    bad.write_text("0 0 0 20 -1 0 : 8 1 16 8\n")
    assert L.hk_tune_load(str(bad).encode(), None) == INVALID
    bad.write_text("0 0 0 20 -1 0 : 12 1 16 8 0\n")  # E_row 12 is not a kernel variant
    assert L.hk_tune_load(str(bad).encode(), None) == INVALID
    assert L.hk_tune_load(str(tmp_path / "missing.txt").encode(), None) == INVALID
    assert L.hk_tune_load(None, None) == NULLP


def test_tensor_matrix_argument_errors(L):
    b = ctypes.c_size_t(0)
    assert L.hankel_tensor_matrix_workspace_size(HK_C64, 1, 8, 2, ctypes.byref(b)) == INVALID
    assert L.hankel_tensor_matrix_workspace_size(HK_C64, 3, 0, 2, ctypes.byref(b)) == INVALID
    assert L.hankel_tensor_matrix_workspace_size(HK_C64, 3, 8, 0, ctypes.byref(b)) == INVALID
    assert L.hankel_tensor_matrix_workspace_size(HK_C64, 5, 8, 64, ctypes.byref(b)) == SIZE  # 64^4 columns
    assert L.hankel_tensor_matrix_workspace_size(HK_C64, 3, 8, 2, None) == NULLP
    assert L.hankel_tensor_matrix(HK_C64, None, 3, 8, 2, None, None, None, 0, None) == NULLP


def test_levels_argument_errors(L):
    b = ctypes.c_size_t(0)
    dims = (ctypes.c_int64 * 6)(4, 3, 2, 5, 2, 3)
    vec = (ctypes.c_void_p * 3)(256, 256, 256)
    f = L.block_hankel_tvp_levels_workspace_size
    assert f(HK_C64, 3, 2, dims, vec, 1, 1, ctypes.byref(b)) == OK and b.value > 0
    assert f(HK_C64, 3, 0, dims, vec, 1, 1, ctypes.byref(b)) == INVALID        # k outside [1, 4]
    assert f(HK_C64, 3, 5, dims, vec, 1, 1, ctypes.byref(b)) == INVALID
    assert f(HK_C64, 1, 2, dims, vec, 1, 1, ctypes.byref(b)) == INVALID        # m outside [2, 8]
    assert f(HK_C64, 3, 2, None, vec, 1, 1, ctypes.byref(b)) == NULLP
    assert f(HK_C64, 3, 2, dims, None, 1, 1, ctypes.byref(b)) == NULLP
    assert f(HK_C64, 3, 2, dims, vec, 0, 0, ctypes.byref(b)) == NULLP          # nothing requested
    big = (ctypes.c_int64 * 6)(3000, 3000, 3000, 3000, 3000, 3000)             # 8998^2 > 2^24 entries
    assert f(HK_C64, 3, 2, big, vec, 1, 1, ctypes.byref(b)) == SIZE
    zero = (ctypes.c_int64 * 6)(4, 0, 2, 5, 2, 3)
    assert f(HK_C64, 3, 2, zero, vec, 1, 1, ctypes.byref(b)) == INVALID
    # the workspace holds the embedded vectors: two distinct ones when mode 1 is not needed
    vec2 = (ctypes.c_void_p * 3)(None, 256, 256)
    b2 = ctypes.c_size_t(0)
    assert f(HK_C64, 3, 2, dims, vec2, 1, 0, ctypes.byref(b2)) == OK and b2.value < b.value


def test_length_policies(L):
    """auto: odd-factor lengths once the power-of-two length reaches 2^18 (one
    product), the factor 5 where the transform is resident (one product of a
    three-pass 5 * 2^18 is too little work for it); pow2: never;
    smallest: always; unknown policies rejected."""
    assert L.hk_get_fft_lengths() == 0
    assert fft_layout(L, 190)[0] == 256 and fft_layout(L, 12000)[0] == 16384
    # 1,100,000 > 2^20: 5 * 2^18 would be three-pass, so auto takes 3 * 2^19
    assert fft_layout(L, 196606)[0] == 3 << 16 and fft_layout(L, 1100000)[0] == 3 << 19
    assert L.hk_set_fft_lengths(1) == OK
    assert fft_layout(L, 196606)[0] == 1 << 18
    assert L.hk_set_fft_lengths(2) == OK
    assert fft_layout(L, 190)[0] == 192 and fft_layout(L, 1100000)[0] == 5 << 18
    assert L.hk_set_fft_lengths(7) == INVALID
    assert L.hk_set_fft_lengths(0) == OK and L.hk_get_fft_lengths() == 0


def test_factor5_block_rows_policy(L):
    """BHHB row axes take 5 * 2^k under auto once instances * grid >= 2^22:
    rows 1228 (inner 410, m = 3) by 511 columns (171 blocks) give 1536 x 512
    for one tensor and 1280 x 512 for a batch of 8 (8 * 1280 * 512 > 2^22)."""
    def grid(policy, batch):
        assert L.hk_set_fft_lengths(policy) == OK
        inner, blocks = (ctypes.c_int64 * 3)(410, 410, 410), (ctypes.c_int64 * 3)(171, 171, 171)
        r, c = ctypes.c_int64(0), ctypes.c_int64(0)
        assert L.block_hankel_tvp_layout(HK_C64, 3, inner, blocks, batch, ctypes.byref(r), ctypes.byref(c)) == OK
        return r.value, c.value
    try:
        assert grid(0, 1) == (1536, 512)
        assert grid(0, 8) == (1280, 512) == grid(2, 8)
        assert grid(1, 8) == (2048, 512)
    finally:
        assert L.hk_set_fft_lengths(0) == OK


def test_factor5_threepass_policy(L):
    """auto takes the three-pass length 5 * 2^14 for d_H = 71,998 (m = 3,
    n = 24,000) once instances * N >= 2^22: a strided batch of 64 sizes its
    workspace as under 'smallest' (same length), a batch of 8 does not; the
    per-instance workspace is N-proportional, so pow2 (2^17) needs more."""
    def ws(policy, batch):
        assert L.hk_set_fft_lengths(policy) == OK
        b = ctypes.c_size_t(0)
        assert L.hankel_tvp_strided_batched_workspace_size(HK_C64, 3, 24000, batch, ctypes.byref(b)) == OK
        return b.value
    try:
        assert ws(0, 64) == ws(2, 64)
        assert ws(0, 8) != ws(2, 8)
        assert ws(1, 64) > ws(0, 64)
    finally:
        assert L.hk_set_fft_lengths(0) == OK


def test_spectral_layout_and_errors(L):
    """The spectral entry points check their arguments on the host."""
    def lay(dt, m, dims):
        n_fft, row = ctypes.c_int64(0), ctypes.c_int64(0)
        d = (ctypes.c_int64 * m)(*dims)
        rc = L.hankel_spectrum_layout(dt, m, d, ctypes.byref(n_fft), ctypes.byref(row))
        return rc, n_fft.value, row.value
    # rows of 2^(ceil(log2 N / 2) + 1) from N = 2^16 on (at most 2^12), else 2^ceil(log2 N / 2)
    assert lay(HK_C64, 4, [1 << 18] * 4) == (OK, 1 << 20, 1 << 11)
    assert lay(HK_C64, 2, [1 << 23] * 2) == (OK, 1 << 24, 1 << 12)
    assert lay(HK_C64, 3, [1 << 15] * 3) == (OK, 1 << 17, 1 << 10)
    assert lay(HK_C128, 3, [3000] * 3) == (OK, 1 << 14, 1 << 7)
    assert lay(HK_C64, 4, [8192] * 4) == (OK, 1 << 15, 1 << 8)
    assert lay(HK_C64, 3, [30] * 3)[0] == NOTSUP      # resident size
    assert lay(HK_F32, 3, [3000] * 3) == (OK, 1 << 14, 1 << 7)    # real dtypes: the complex layout
    assert lay(9, 3, [3000] * 3)[0] == INVALID
    assert lay(HK_C64, 1, [3000])[0] == INVALID
    assert lay(HK_C64, 3, [3000, 0, 5])[0] == INVALID
    d = (ctypes.c_int64 * 3)(3000, 3000, 3000)
    b = ctypes.c_size_t(0)
    assert L.hankel_spectrum_workspace_size(HK_C64, 3, d, 3, ctypes.byref(b)) == INVALID
    assert L.hankel_spectrum_workspace_size(HK_C64, 3, d, -2, ctypes.byref(b)) == INVALID
    assert L.hankel_spectrum_workspace_size(HK_C64, 3, d, -1, ctypes.byref(b)) == OK
    assert b.value >= (1 << 14) * 8
    assert L.hankel_spectrum(HK_C64, 3, d, -1, None, ctypes.c_void_p(256), ctypes.c_void_p(256), b.value,
                             None) == NULLP
    assert L.hankel_spectrum(HK_C64, 3, d, -1, ctypes.c_void_p(260), ctypes.c_void_p(256), ctypes.c_void_p(256),
                             b.value, None) == MISALIGNED
    # products: h spectrum missing, a vector missing, too small a workspace
    v = (ctypes.c_void_p * 3)(256, 512, 768)
    assert L.hankel_mode_products_spectral_workspace_size(HK_C64, 3, d, v, None, 1, 0, ctypes.byref(b)) == OK
    need = b.value
    assert L.hankel_mode_products_spectral(HK_C64, None, 3, d, v, None, ctypes.c_void_p(256), None,
                                           ctypes.c_void_p(256), need, None) == NULLP
    v0 = (ctypes.c_void_p * 3)(256, None, 768)
    assert L.hankel_mode_products_spectral(HK_C64, ctypes.c_void_p(256), 3, d, v0, None, ctypes.c_void_p(256), None,
                                           ctypes.c_void_p(256), need, None) == NULLP
    assert L.hankel_mode_products_spectral(HK_C64, ctypes.c_void_p(256), 3, d, v, None, ctypes.c_void_p(256), None,
                                           ctypes.c_void_p(256), need - 1, None) == WORKSPACE
    # every operand a spectrum: one output buffer and the partial sums only
    s = (ctypes.c_void_p * 3)(1024, 1280, 1536)
    assert L.hankel_mode_products_spectral_workspace_size(HK_C64, 3, d, None, s, 1, 1, ctypes.byref(b)) == OK
    assert b.value < need


def test_spectral_batch_argument_errors(L):
    b = ctypes.c_size_t(0)
    assert L.hankel_tvp_spectral_strided_batched_workspace_size(HK_C64, 4, 1 << 14, 8, ctypes.byref(b)) == OK
    one = ctypes.c_size_t(0)
    assert L.hankel_tvp_spectral_strided_batched_workspace_size(HK_C64, 4, 1 << 14, 1, ctypes.byref(one)) == OK
    assert b.value == 8 * one.value
    assert L.hankel_tvp_spectral_strided_batched_workspace_size(HK_C64, 4, 1 << 14, -1, ctypes.byref(b)) == INVALID
    assert L.hankel_tvp_spectral_strided_batched_workspace_size(HK_F64, 4, 1 << 14, 8, ctypes.byref(b)) == OK
    assert L.hankel_tvp_spectral_strided_batched_workspace_size(HK_C64, 3, 100, 8, ctypes.byref(b)) == NOTSUP
    P = ctypes.c_void_p
    assert L.hankel_tvp_spectral_strided_batched(HK_C64, None, 4, 1 << 14, P(256), 1 << 14, P(256), 1 << 14, None, 8,
                                                 P(256), 8 * one.value, None) == NULLP
    assert L.hankel_tvp_spectral_strided_batched(HK_C64, P(256), 4, 1 << 14, P(256), 1 << 14, P(256), 1 << 14, None, 8,
                                                 P(256), 8 * one.value - 1, None) == WORKSPACE


def test_spectral_layout_ignores_length_policy(L):
    """Stored spectra keep the power-of-two layout under every length policy
    (d_H = 196606 would take 3 * 2^16 under 'smallest'), so spectra made under
    different policies still combine."""
    def lay(m, dims):
        n_fft, row = ctypes.c_int64(0), ctypes.c_int64(0)
        d = (ctypes.c_int64 * m)(*dims)
        assert L.hankel_spectrum_layout(HK_C64, m, d, ctypes.byref(n_fft), ctypes.byref(row)) == OK
        return n_fft.value, row.value
    try:
        for policy in (0, 1, 2):
            assert L.hk_set_fft_lengths(policy) == OK
            assert lay(3, [65536] * 3) == (1 << 18, 1 << 10)
    finally:
        assert L.hk_set_fft_lengths(0) == OK


def test_spectral_batch_of_zero(L):
    """An empty strided spectral batch succeeds on the host without the device."""
    P = ctypes.c_void_p
    assert L.hankel_tvp_spectral_strided_batched(HK_C64, P(256), 4, 1 << 14, P(256), 1 << 14, P(256), 1 << 14, None, 0,
                                                 None, 0, None) == OK


def _problem(is_block):
    q = _lib.hk_problem_t()
    q.m = 3
    q.is_block = is_block
    for k in range(3):
        q.dims[k] = 40
        q.block_dims[k] = 30 if is_block else 0
        q.vectors[k] = 0x10000 * (k + 1)
    q.h = 0x100000
    q.y = 0x200000
    return q


@pytest.mark.parametrize("fn,bad", [("hankel_mode_products_batched", 1), ("block_hankel_tvp_batched", 0)])
def test_kind_restricted_batches_reject_the_other_kind(L, fn, bad):
    """A problem of the other kind is rejected before any device work, in the
    workspace query and in the call (every pointer here is a host-side dummy)."""
    arr = (_lib.hk_problem_t * 2)(_problem(1 - bad), _problem(bad))
    b = ctypes.c_size_t(0)
    assert getattr(L, fn + "_workspace_size")(HK_C64, arr, 2, ctypes.byref(b)) == INVALID
    assert getattr(L, fn)(HK_C64, arr, 2, ctypes.c_void_p(0x400000), 1 << 20, None) == INVALID
    assert b"BHHB" in L.hk_last_error()
    assert getattr(L, fn + "_workspace_size")(HK_C64, None, 1, ctypes.byref(b)) == NULLP


def _mixed_problem_array(count=512, seed=11):
    """Host-side descriptors with dummy (aligned, never dereferenced) device
    pointers: orders 3..5, d_H from a few hundred to ~80 k, equal and
    distinct vectors."""
    import numpy as np
    g = np.random.Generator(np.random.PCG64(seed))
    arr = (_lib.hk_problem_t * count)()
    base = 1 << 30
    for i in range(count):
        q = arr[i]
        q.m = int(g.integers(3, 6))
        n = int(np.exp(g.uniform(np.log(64), np.log(16384))))
        equal = bool(g.integers(0, 2))
        for k in range(q.m):
            q.dims[k] = n
            if k > 0:
                q.vectors[k] = base + (256 if equal else 256 * k)
        q.h = base + 4096
        q.y = base + 8192
        base += 1 << 20
    return arr


def test_autotune_workspace_covers_every_candidate(L):
    """HK_PLAN_AUTOTUNE may rebuild any length bucket with powers of two or
    without the factor 5: its workspace query must cover the default plan and
    the all-powers-of-two plan (the plans need no device to be built)."""
    arr = _mixed_problem_array()

    def ws_of(flags):
        plan = ctypes.c_void_p()
        assert L.hk_plan_create(ctypes.byref(plan), HK_C64, arr, len(arr), flags) == OK, L.hk_last_error()
        b = ctypes.c_size_t(0)
        assert L.hk_plan_workspace_size(plan, ctypes.byref(b)) == OK
        assert L.hk_plan_destroy(plan) == OK
        return b.value

    grouped = _lib.HK_PLAN_MULTIKERNEL
    tuned = ws_of(grouped | _lib.HK_PLAN_AUTOTUNE)
    assert tuned >= ws_of(grouped)
    assert tuned >= ws_of(grouped | _lib.HK_PLAN_POW2)
    # graph plans are not tuned: no extra workspace
    assert ws_of(grouped | _lib.HK_PLAN_AUTOTUNE | _lib.HK_PLAN_GRAPH) == ws_of(grouped | _lib.HK_PLAN_GRAPH)
