"""MI355X-native open-boundary ballistic transport solver.

The HIP library (libqtx.so, C ABI in include/qtx.h) is loaded lazily by
`paper_1903_00548_amd._lib.load()`; importing this package does not touch
the GPU.  `workloads` holds the seeded synthetic inputs.
"""
__all__ = ["workloads", "_lib"]
