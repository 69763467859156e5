"""qpt: progressive quasi-Monte Carlo path tracing on MI355X (gfx950).

The hot path lives in libqpt.so (HIP kernels + C-ABI, declared in
include/qpt.h); :mod:`paper_1705_01263_amd.qpt` is the thin ctypes binding.
"""
from .qpt import Context, Renderer, QptError, lib  # noqa: F401
