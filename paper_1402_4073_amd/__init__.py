"""Threshold and symmetric queries over bitmaps, native to AMD MI355X (gfx950).

The computation lives in libtq.so (HIP kernels behind a C ABI, declared in
include/tq.h); ``binding`` forwards to it with the same function names.
"""
from . import binding  # noqa: F401
from .binding import (Context, TQError, tq_create, tq_ctx_check, tq_destroy,  # noqa: F401
                      tq_symmetric, tq_threshold)
