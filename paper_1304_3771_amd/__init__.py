"""MI355X (gfx950) guest-memory translate-and-copy library.

The work is done by libdevirt.so (HIP kernels behind the C ABI of
include/devirt.h); this package only marshals arguments to it.
"""
from .devirt import (  # noqa: F401
    CODES,
    COMPLETION_DTYPE,
    EPT_MAP_DTYPE,
    EPT_R,
    EPT_W,
    EPT_X,
    FAULT_DTYPE,
    FROM_GUEST,
    MAP_DTYPE,
    MAP_WRITE,
    REQUEST_DTYPE,
    RESULT_DTYPE,
    TO_GUEST,
    XLAT_DTYPE,
    XLAT_SET_AD,
    XLAT_WRITE,
    Context,
    DevirtError,
    Server,
    header_functions,
    lib,
)
