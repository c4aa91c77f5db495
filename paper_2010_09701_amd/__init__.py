"""MI355X (gfx950) HIP library for the Chebyshev-filtered subspace iteration on the
orthogonalized-enriched finite-element Kohn-Sham operator (arXiv 2010.09701).

Submodules (imported lazily so that input generation works without a device):
  workloads  seeded synthetic systems and random blocks
  oefe       ctypes binding of liboefe.so (the C ABI in include/oefe.h)
  chfsi      ChFSI pass driver
  autograd   torch.autograd.Function for the band energy
  build      in-tree build of liboefe.so for gfx950
"""
