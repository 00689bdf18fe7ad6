"""Host-side checks of the Python binding (no GPU): every entry point rejects
tensors whose size, dtype or device does not match the shape of the call
before anything reaches the library, and autograd cotangents that arrive as
lazy conjugate / negative views are materialized first."""
import pytest
import torch

from paper_1401_6238_amd import _lib, binding

HOST_ONLY = {"hankel_spectrum_layout"}


class _NoDeviceCalls:
    """Stands in for libhankel.so: host-only queries go to the real library,
    any other call fails the test (validation must come first)."""

    def __getattr__(self, name):
        if name in HOST_ONLY:
            return getattr(_lib.lib(), name)
        raise AssertionError(f"library entry point {name} reached with invalid arguments")


@pytest.fixture
def B(monkeypatch):
    def dev_on_host(t):
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if t.is_conj() or t.is_neg():
            raise ValueError("pending conjugation")
        return t
    monkeypatch.setattr(binding, "_dev", dev_on_host)
    monkeypatch.setattr(binding, "lib", lambda: _NoDeviceCalls())
    return binding


C = torch.complex64


def z(n, dtype=C):
    return torch.zeros(n, dtype=dtype)


def test_tvp_rejects_wrong_h_length(B):
    with pytest.raises(ValueError, match="h has 9 elements, expected 10"):
        B.hankel_tvp(z(9), z(4), 3)
    with pytest.raises(TypeError, match="dtype"):
        B.hankel_tvp(z(10, torch.complex128), z(4), 3)


def test_mode_products_rejects(B):
    with pytest.raises(ValueError, match="h has"):
        B.hankel_mode_products(z(6), [z(3), z(4), z(2)], want_alpha=True)   # d_H = 3 + 4 + 2 - 3 + 1 = 7
    with pytest.raises(ValueError, match=r"vectors\[1\]"):
        B.hankel_mode_products(z(7), [None, z(5), z(2)], dims=[3, 4, 2])
    with pytest.raises(ValueError, match=r"vectors\[0\] is needed"):
        B.hankel_mode_products(z(7), [None, z(4), z(2)], dims=[3, 4, 2], want_alpha=True)


def test_block_rejects(B):
    # inner (2, 3), blocks (4, 2): H is (2+3-1) x (4+2-1) = 4 x 5
    with pytest.raises(ValueError, match="H has 19 elements, expected 20"):
        B.block_hankel_tvp(z(19), [None, z(6)], [2, 3], [4, 2])
    with pytest.raises(ValueError, match=r"vectors\[1\] has 5"):
        B.block_hankel_tvp(z(20), [None, z(5)], [2, 3], [4, 2])


def test_levels_rejects(B):
    with pytest.raises(ValueError, match="G has"):
        B.block_hankel_tvp_levels(z(10), [None, z(6)], [[2, 3], [4, 2]])


def test_backward_rejects(B):
    m, n = 3, 5
    h, x = z(m * (n - 1) + 1), z(n)
    with pytest.raises(ValueError, match="h has"):
        B.hankel_tvp_backward(z(12), x, m, z(n), None)
    with pytest.raises(ValueError, match="grad_y has 4"):
        B.hankel_tvp_backward(h, x, m, z(4), None)
    with pytest.raises(ValueError, match="grad_alpha has 2"):
        B.hankel_tvp_backward(h, x, m, None, z(2))
    with pytest.raises(TypeError, match="grad_y has dtype"):
        B.hankel_tvp_backward(h, x, m, z(n, torch.complex128), None)


def test_backward_spectral_rejects(B):
    m, n = 3, 4096                      # d_H = 12286 -> N = 16384
    h = z(m * (n - 1) + 1)
    with pytest.raises(ValueError, match="h has"):
        B.hankel_tvp_backward_spectral(z(100), z(16384), m, n, z(n), None)
    with pytest.raises(ValueError, match="x_spec has 8192"):
        B.hankel_tvp_backward_spectral(h, z(8192), m, n, z(n), None)
    with pytest.raises(TypeError, match="x_spec has dtype"):
        B.hankel_tvp_backward_spectral(h, z(16384, torch.complex128), m, n, z(n), None)


def test_spectral_rejects(B):
    m, n = 3, 4096
    dims = [n] * m
    with pytest.raises(ValueError, match="src has"):
        B.hankel_spectrum(z(n - 1), m, dims, 1)
    with pytest.raises(ValueError, match="h_spec has"):
        B.hankel_mode_products_spectral(z(100), m, dims, vectors=[None, z(n), z(n)])
    with pytest.raises(ValueError, match=r"specs\[2\] has"):
        B.hankel_mode_products_spectral(z(16384), m, dims, vectors=[None, z(n), None],
                                        specs=[None, None, z(10)], dtype=C)
    with pytest.raises(ValueError, match="h_spec has"):
        B.hankel_tvp_spectral_strided_batched(z(100), torch.zeros(2, n, dtype=C), m)


def test_strided_rejects(B):
    m, n, b = 3, 6, 2
    with pytest.raises(ValueError, match="h has"):
        B.hankel_tvp_strided_batched(torch.zeros(b, 15, dtype=C), torch.zeros(b, n, dtype=C), m)
    h, x = torch.zeros(b, 16, dtype=C), torch.zeros(b, n, dtype=C)
    with pytest.raises(ValueError, match="grad_y has"):
        B.hankel_tvp_backward_strided_batched(h, x, m, torch.zeros(b, n - 1, dtype=C), None)
    with pytest.raises(ValueError, match="grad_alpha has"):
        B.hankel_tvp_backward_strided_batched(h, x, m, None, torch.zeros(b + 1, dtype=C))
    with pytest.raises(ValueError, match="H has"):
        B.block_hankel_tvp_strided_batched(torch.zeros(b, 10, dtype=C), torch.zeros(b, 6, dtype=C), 3, 2, 3)


def test_plan_rejects(B):
    probs = [dict(m=3, dims=[4, 4, 4], h=z(9), vectors=[None, z(4), z(4)])]
    with pytest.raises(ValueError, match="problem 0 h has 9"):
        B.Plan(probs)
    probs = [dict(m=2, dims=[4, 3], h=z(6), vectors=[None, z(4)])]
    with pytest.raises(ValueError, match=r"problem 0 vectors\[1\] has 4"):
        B.Plan(probs)


def test_tensor_matrix_rejects(B):
    with pytest.raises(ValueError, match="h has"):
        B.hankel_tensor_matrix(z(10), torch.zeros(5, 2, dtype=C), 3)


def test_cotangent_conj_view_is_materialized(B):
    v = torch.tensor([1 + 2j, 3 - 1j, -2 + 0.5j], dtype=C)
    lazy = v.conj()
    assert lazy.is_conj()
    got = B._cotangent(lazy, "grad_y", 3, C, v.device)
    assert not got.is_conj()
    assert torch.equal(got, torch.conj_physical(v))
    neg = torch.neg(v.conj()).conj()   # a lazy negative view on some builds; values -v either way
    got = B._cotangent(neg, "grad_y", 3, C, v.device)
    assert not got.is_neg() and not got.is_conj()
    assert torch.equal(got, -v)


def test_batched_oneshot_rejects(B):
    with pytest.raises(ValueError, match="problem 0: no vector given"):
        B.hankel_mode_products_batched([dict(m=2, dims=[4, 3], h=z(6), vectors=[None, None])])
    probs = [dict(m=3, dims=[4, 4, 4], h=z(9), vectors=[None, z(4), z(4)])]
    with pytest.raises(ValueError, match="problem 0 h has 9"):
        B.block_hankel_tvp_batched(probs)
