"""MI355X (gfx950) checkerboard Metropolis engine for the 2D Ising model.

The compute path is the HIP library ``libising_mi355x.so`` behind the C ABI
in ``include/ising.h``; ``binding`` is a thin ctypes layer over it with the
same function names. Importing this package does not load the library; the
first call that needs it does, and raises if it is missing (there is no CPU
fallback).
"""

__all__ = ["binding", "workloads"]
