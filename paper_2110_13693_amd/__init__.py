"""MI355X (gfx950) evaluator of warehouse picking plans.

The compute path is ``libwo.so`` (hand-written HIP kernels behind the C ABI
of ``include/wo.h``); :mod:`.wo` is a thin ctypes binding with the same names.
PyTorch only provides device memory and streams.
"""
from . import wo  # noqa: F401
