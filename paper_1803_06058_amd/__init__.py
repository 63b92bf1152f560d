"""LOVE (LanczOs Variance Estimates) for KISS-GP on AMD Instinct MI355X.

Thin Python binding over the native C ABI in ``include/love.h`` (library
``_lib/liblove.so``).  Every step of the method runs in the library's HIP
kernels; this package only marshals torch device tensors (pointers, sizes,
the current stream) into the C calls.  There is no CPU fallback: importing
the binding without a built library raises.
"""
from .binding import (  # noqa: F401
    LoveError, LoveCache, build_cache, build_cache_batched, predict_mean_var_batched,
    lib_path, load_library, profile_enable, profile_read, profile_select, LovePredict, config_struct,
    PRECISIONS, KERNELS, TOEPLITZ_MODES,
)
