"""MI355X-native third-order relativistic lattice Boltzmann (RLBD).

The compute path is the C-ABI library ``librlb.so`` (HIP kernels for
gfx950) declared in ``include/rlb.h``; ``paper_1301_3423_amd.rlb`` is its
thin ctypes binding.  Nothing is loaded at import time: the library is
opened on first use, and a missing library raises instead of falling back.
"""
__all__ = ["rlb", "inputs"]
