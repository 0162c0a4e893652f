"""MI355X-native engine for iterated Jacobi stencil sweeps under deep temporal blocking.

The compute path lives in ``libstencil.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/stencil.h``). ``paper_2305_07390_amd.stencil`` is a
thin ctypes binding with the same entry-point names; it loads the library on
first use and raises if the library is missing.
"""

__all__ = ["stencil", "workloads"]
