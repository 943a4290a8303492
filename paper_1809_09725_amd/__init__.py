"""MI355X-native decomposed-time 4D tomography (Nikitin et al.): the
decomposed-time Radon operator R_T, its adjoint, the 4D TV steps and the
adapted Chambolle-Pock solver, as HIP kernels for gfx950 behind the C ABI
of include/rt4d.h.

Submodules:
  rt4d     ctypes binding of librt4d.so (Plan, Job and the C-named calls)
  serving  continuous-batching request loop over the job API
  inputs   seeded synthetic phantoms and operands
  build    compiles librt4d.so in-tree with hipcc
"""
