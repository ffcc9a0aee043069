"""MI355X-native polyharmonic-spline interpolation (hand-written HIP for gfx950).

The compute path lives in libphs.so (csrc/*.hip) behind the C ABI declared in
include/phs.h; `native` is the ctypes binding that hands torch device pointers
and the current stream to it.  `workloads` draws the seeded synthetic inputs.
"""
__all__ = ["native", "workloads", "build"]
