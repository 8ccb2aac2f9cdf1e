"""Square-root bundle adjustment on one AMD MI355X (gfx950).

The solver lives in the HIP/C++ library ``libsqrtba.so`` (C ABI:
``include/sqrtba.h``); ``sqrtba`` is its thin ctypes binding.
"""

from .sqrtba import (  # noqa: F401
    Context,
    Options,
    Report,
    SqrtBAError,
    default_options,
    lib,
    LIB_PATH,
    EXPORTED,
)
