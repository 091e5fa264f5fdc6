"""MI355X (gfx950) streaming method-of-snapshots DMD.

The compute path is the HIP library libdmdstream.so (C ABI in
include/dmd_stream.h); this package is its Python binding.  Build the library
with ``python -m paper_1612_07875_amd.build``.
"""

from .binding import (
    Stream, Batch, DMDError, load, last_error, LIB_PATH, SIGNATURES, STRING_FUNCS,
    footprint, make_opts, window_gram, tune, tune_lookup, tune_save, tune_load, tune_clear, profile_enable, profile_reset, profile_read,
    OK, W_RANK, E_INVAL, E_NOMEM, E_NOT_READY, E_NONFINITE, E_CONVERGENCE, E_DEVICE, E_UNSUPPORTED,
)

__all__ = [
    "Stream", "Batch", "DMDError", "load", "last_error", "LIB_PATH", "SIGNATURES", "STRING_FUNCS",
    "footprint", "make_opts", "window_gram", "tune", "tune_lookup", "tune_save", "tune_load", "tune_clear",
    "profile_enable", "profile_reset", "profile_read",
    "OK", "W_RANK", "E_INVAL", "E_NOMEM", "E_NOT_READY", "E_NONFINITE", "E_CONVERGENCE",
    "E_DEVICE", "E_UNSUPPORTED",
]
