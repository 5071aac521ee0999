"""CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (plain sequential C) with ctypes.
"""
from .oracle import (  # noqa: F401
    CODES,
    FAULT_DTYPE,
    RESULT_DTYPE,
    XLAT_DTYPE,
    Oracle,
    build,
)
