"""Digital Voronoi, Laguerre and Johnson-Mehl diagrams on MI355X.

The labelling runs in the HIP kernels of ``libvtess.so`` behind the C ABI of
``include/vtess.h``; ``vtess`` is its ctypes binding, ``serve`` the
continuous-batching request loop and ``inputs`` the seeded synthetic
workloads.  Importing the package loads nothing; the library is loaded on
first use and its absence is an error.
"""
__all__ = ["vtess", "serve", "inputs"]
