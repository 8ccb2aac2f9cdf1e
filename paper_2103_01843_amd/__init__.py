"""Square-root bundle adjustment on one AMD MI355X (gfx950).

The solver lives in the HIP/C++ libraries ``libsqrtba.so`` (FP32, C ABI
``include/sqrtba.h``) and ``libsqrtba64.so`` (FP64, ``include/sqrtba64.h``);
``sqrtba`` is their thin ctypes binding (``Context(precision=64)`` selects the
FP64 one).
"""

from .sqrtba import (  # noqa: F401
    Context,
    Options,
    Report,
    SqrtBAError,
    default_options,
    lib,
    LIB_PATH,
    LIB64_PATH,
    EXPORTED,
    EXPORTED64,
)
