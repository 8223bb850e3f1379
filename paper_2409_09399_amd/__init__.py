"""MI355X-native grid integration (Gint) for numerical-atomic-orbital DFT.

Submodules:
  inputs  seeded synthetic workloads (no grid-integration arithmetic)
  gint    ctypes binding of the HIP library libgint.so (C ABI in include/gint.h)
"""
