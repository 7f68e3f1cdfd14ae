"""mdseries for MI355X: one Newton step on truncated power series in complex
multiple-double precision (arXiv:2012.06607), as hand-written HIP kernels
behind a C ABI (include/mdseries.h).

Submodules:
  binding  ctypes binding of libmdseries.so (torch tensors in, no arithmetic)
  inputs   seeded synthetic inputs (exact rationals rounded to limbs)
  build    compiles the HIP sources into libmdseries.so
"""
