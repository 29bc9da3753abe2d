"""MI355X-native staggered-leapfrog lattice evolution of classical scalar fields.

The compute path is the C-ABI library ``libce.so`` (hand-written HIP kernels
for gfx950); ``paper_0712_0813_amd.ce`` is its thin ctypes binding.  Importing
this package does not load the library.
"""
__all__ = ["ce", "inputs", "workloads"]
