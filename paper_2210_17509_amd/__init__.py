"""MI355X-native GRMHD hot path (GRaM-X, arXiv:2210.17509): HIP kernels behind a C ABI.

Submodules:
  inputs  seeded synthetic problems (no method arithmetic)
  build   hipcc build of libgrmhd.so
  grmhd   ctypes binding of the C ABI (imports only when the library is built)
"""
