"""MI355X-native relativistic lattice Boltzmann (RLBM) collide-and-stream library.

The compute path is ``librlbm.so`` (hand-written HIP for gfx950) behind the C
ABI of ``include/rlbm.h``; ``paper_1909_04502_amd.rlbm`` is its ctypes binding.
"""
from .rlbm import Batch, Lattice, RLBMError, lib, quadrature_build  # noqa: F401
