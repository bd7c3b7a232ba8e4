"""MI355X (gfx950) SsNAL-EN elastic-net solver.

The solver lives in the HIP library libssnal_en.so (C ABI in
include/ssnal_en.h); `paper_2006_03970_amd.binding` exposes its entry points
to Python.  Importing this package does not load the library.
"""
__all__ = ["binding", "build"]
