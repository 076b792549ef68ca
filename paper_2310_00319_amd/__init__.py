"""MI355X-native TVOLAP (Time-Variant Overlap-Add in Partitions).

The compute path is the gfx950 HIP library ``libtvolap.so`` (C ABI in
``include/tvolap.h``); this package only marshals arguments to it.
"""
from .convolver import Convolver  # noqa: F401
from ._lib import TvolapError, load  # noqa: F401
from . import functional  # noqa: F401

__all__ = ["Convolver", "TvolapError", "load", "functional"]
