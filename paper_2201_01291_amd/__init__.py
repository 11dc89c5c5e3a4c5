"""MI355X-native vertex-centred explicit residual (AVIP method, arXiv 2201.01291).

Submodules:
  workloads  seeded synthetic meshes and initial states (inputs only)
  vcx        ctypes binding of the HIP library libvcx.so (include/vcx.h)
  build      compiles libvcx.so for gfx950
"""
