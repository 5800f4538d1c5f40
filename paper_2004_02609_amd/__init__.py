"""MI355X (gfx950) FFT-accelerated capacitance extraction for voxelized structures.

The solver is the HIP library libvoxcap.so behind the C ABI of include/voxcap.h;
`voxcap` is its ctypes binding.
"""
from . import voxcap  # noqa: F401
from .voxcap import Problem, VoxcapError  # noqa: F401
