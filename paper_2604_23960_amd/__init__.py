"""MI355X-native multi-robot motion validation: MotionValidation (MV) and
FindFirstConflict (FFC) as HIP kernels behind a C ABI (include/mrv.h).

``mrv`` is the ctypes binding, ``workloads`` the seeded synthetic inputs and
``build`` compiles libmrv.so for gfx950.
"""
__all__ = ["mrv", "workloads", "build"]
