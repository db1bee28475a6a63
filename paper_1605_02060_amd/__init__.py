"""Masked LDDMM registration on AMD MI355X (HIP kernels behind a C ABI).

Submodules:
  lddmm  -- ctypes binding of liblddmm.so (the product path; GPU only)
  synth  -- seeded synthetic workloads
  build  -- builds liblddmm.so in-tree with hipcc
"""
