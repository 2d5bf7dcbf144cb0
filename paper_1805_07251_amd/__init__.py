"""MI355X (gfx950) implementation of the multicomponent van der Waals
free-energy lattice Boltzmann sweep of Ridl & Wagner (arXiv:1805.07251).

Modules
  vdwlb     ctypes binding of libvdwlb.so (the C-ABI of include/vdwlb.h)
  lattice   Plan / Lattice: one periodic D2Q9 lattice on the GPU
  inputs    seeded synthetic workloads (no lattice Boltzmann arithmetic)
  build     in-tree hipcc build of libvdwlb.so
"""
from . import inputs, vdwlb  # noqa: F401

__all__ = ["inputs", "vdwlb"]
