"""Fast Hankel tensor-vector products on MI355X (gfx950).

The arithmetic runs in libhankel.so (hand-written HIP kernels); this package
marshals torch tensors to its C ABI.  Importing the package does not load the
library; the first call does, and raises if it has not been built.
"""
__all__ = [
    "hankel_tvp", "hankel_mode_products", "hankel_spectrum_layout", "hankel_spectrum", "hankel_mode_products_spectral", "hankel_tvp_spectral_strided_batched", "hankel_tvp_backward_spectral", "hankel_tvp_save_spectrum", "hankel_tvp_backward_spectral_strided_batched", "hankel_tvp_noalloc", "block_hankel_tvp", "block_hankel_tvp_layout", "block_hankel_tvp_levels", "hankel_tvp_backward",
    "hankel_tvp_strided_batched", "hankel_tvp_backward_strided_batched", "block_hankel_tvp_strided_batched",
    "hankel_tvp_batched", "Plan", "hk_fft_layout", "hk_set_fft_lengths", "hk_get_fft_lengths", "hankel_tensor_matrix", "hk_autotune_tvp", "hk_autotune", "hk_tune_save", "hk_tune_load", "hk_last_launch_count", "hk_profile_start", "hk_profile_stop",
    "hankel_mode_products_backward", "block_hankel_tvp_backward", "hankel_mode_products_batched",
    "block_hankel_tvp_batched",
    "HankelTVPFunction", "hankel_tvp_autograd", "HankelModeProductsFunction", "hankel_mode_products_autograd",
    "BlockHankelTVPFunction", "block_hankel_tvp_autograd",
]


def __getattr__(name):
    if name in ("HankelTVPFunction", "hankel_tvp_autograd", "HankelModeProductsFunction",
                "hankel_mode_products_autograd", "BlockHankelTVPFunction", "block_hankel_tvp_autograd"):
        from . import autograd
        return getattr(autograd, name)
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
