"""MI355X (gfx950) implementation of the pseudo-potential lattice Boltzmann
update of arXiv 2504.15018, behind the C ABI of libplbm (include/plbm.h).

  native    ctypes binding, one function per C entry point
  lattice   Lattice: a handle plus its PyTorch-owned device buffer
  serving   continuous-batching request loop over plbm_batch_*
  build     in-tree hipcc build of libplbm.so for gfx950
"""
