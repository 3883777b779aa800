"""MI355X (gfx950) implementation of the per-particle step of the
charge-conserving PIC scheme with alternating-order interpolation
(Sokolov, arXiv:1101.0809).

The compute path is the HIP library ``libpic.so`` (C ABI in include/pic.h);
``Sim`` is a thin PyTorch-backed front end that owns device buffers and
passes pointers.
"""
from ._lib import PicError, load as load_library  # noqa: F401

__all__ = ["Sim", "PicError", "load_library"]


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    raise AttributeError(name)
