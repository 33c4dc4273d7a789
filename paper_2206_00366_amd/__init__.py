"""MI355X-native rectangular MRT lattice Boltzmann (RMRT-LB) hot path.

The compute path is librmrt.so (hand-written HIP kernels for gfx950 behind the
C ABI of include/rmrt.h); `paper_2206_00366_amd.rmrt` is its ctypes binding.
Build it with `python -m paper_2206_00366_amd.build`.
"""
__all__ = ["rmrt"]
