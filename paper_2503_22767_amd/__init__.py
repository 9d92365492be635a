"""MI355X-native magneto-elastic MLS-MPM rollout and adjoint.

Submodules (imported on demand so that the input generator stays free of the
HIP library):
  workloads  seeded synthetic inputs (no simulation arithmetic)
  mpm_mag    ctypes binding of include/mpm_mag.h and the autograd Function
  build      hipcc build of libmpm_mag.so for gfx950
"""
