"""MI355X-native DEM contact pipeline (binning, neighbour list with tangential
history, damped Hertz contact forces with the Coulomb cap, velocity Verlet).

The compute path is the HIP library ``libdem.so`` behind the C-ABI declared in
``include/dem.h``; ``paper_1705_03850_amd.dem`` is the thin ctypes binding.
Submodules are imported lazily so that the input generators can be used
without loading the GPU library.
"""
__all__ = ["dem", "inputs"]
