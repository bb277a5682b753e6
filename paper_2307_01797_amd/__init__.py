"""MI355X-native Ito-KMC particle-mesh step (gfx950 HIP kernels behind a C ABI).

The compiled library is loaded lazily by :mod:`paper_2307_01797_amd.itokmc`; importing
this package (e.g. for :mod:`paper_2307_01797_amd.workloads`) does not touch the GPU.
"""
__all__ = ["workloads", "itokmc"]
