"""mdeos: MI355X-native in-line molecular-dynamics equation of state.

The compute path is the HIP library ``libmdeos.so`` (kernels for gfx950 behind
a C ABI declared in ``include/mdeos.h``); ``paper_2508_06012_amd.mdeos`` is a
thin ctypes binding with the same entry-point names. Importing this package
does not load the library; the binding loads it on first use and raises if it
is missing.
"""
__all__ = ["mdeos", "workloads"]
