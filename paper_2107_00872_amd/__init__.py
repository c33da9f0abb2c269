"""MI355X-native engine for the XXZ model near saturation (QS^3, arXiv 2107.00872).

The compute path is libqs3.so (HIP for gfx950) behind the C ABI of
include/qs3.h; ``qs3`` is its Python binding.
"""
from . import qs3  # noqa: F401
from .qs3 import Batch, Context, Lattice, Sector, Server  # noqa: F401
