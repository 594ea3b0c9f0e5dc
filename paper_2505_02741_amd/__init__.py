"""dyGRASS update path on MI355X: device-resident dynamic adjacency and
batched non-backtracking walks behind the C ABI of include/dygrass.h.

Submodules:
  dygrass    ctypes binding of libdygrass.so (same names as the C ABI)
  workloads  seeded synthetic graphs, sparsifiers and update streams
  build      hipcc build of libdygrass.so for gfx950
"""
