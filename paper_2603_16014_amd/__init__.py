"""MI355X-native fast multitask Gaussian-process likelihood (HIP, gfx950).

The compute path is the C ABI of ``include/mtgp.h`` implemented by
``libmtgp.so`` (hand-written HIP kernels); this package only marshals
arguments to it (``mtgp``) and wraps it for autograd and optimisation
(``training``).  There is no CPU fallback.
"""
from . import _lib  # noqa: F401

__all__ = ["mtgp", "training"]
