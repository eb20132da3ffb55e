"""Exact decimal -> binary64/binary32 parsing on AMD Instinct MI355X.

The parser itself is libffp.so (HIP kernels for gfx950 behind the C-ABI of
include/ffp.h); this package holds its sources, its build step and a thin
ctypes binding.
"""

from . import ffp  # noqa: F401
from .ffp import (  # noqa: F401
    Context,
    FFPError,
    FFP_INVALID,
    FFP_OK,
    FFP_OUT_OF_RANGE,
    load,
)
