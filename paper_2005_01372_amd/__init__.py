"""MI355X-native preconditioned Lippmann-Schwinger solver (HIP kernels behind a C ABI).

The compiled library is loaded lazily by :mod:`paper_2005_01372_amd.lsop`, so
importing the package (or its input generators) never touches the GPU.
"""
__all__ = ["lsop", "synth"]
