"""MI355X (gfx950) neural loss-recovery forward pass of ReVo (arXiv 2604.27441).

The work runs in ``librevo.so`` (hand-written HIP kernels behind a C ABI,
``include/revo.h``).  This package is a thin ctypes binding: it marshals
arguments and uses PyTorch only for device memory and streams.  Importing
it fails loudly when the library has not been built.
"""
from ._lib import lib, LIB_PATH, RevoError, check
from .api import Recoverer, Trainer, Completion, REVO_FP32, REVO_BF16, REVO_FP8

__all__ = ["lib", "LIB_PATH", "RevoError", "check", "Recoverer", "Trainer", "Completion", "REVO_FP32", "REVO_BF16", "REVO_FP8"]
