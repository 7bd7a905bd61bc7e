"""MI355X-native adaptive-relaxation lattice Boltzmann solver.

The compute path is the HIP library ``libarlbm.so`` (C ABI, declared in
``include/arlbm.h``); ``paper_2609_18177_amd.arlbm`` is its thin ctypes
binding.  Importing this package loads nothing: the binding loads the library
on first use and raises if it is missing.
"""
__all__ = ["workloads"]
