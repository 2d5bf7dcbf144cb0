"""MI355X (gfx950) implementation of the multicomponent van der Waals
free-energy lattice Boltzmann sweep of Ridl & Wagner (arXiv:1805.07251).

Modules
  vdwlb         ctypes binding of libvdwlb.so (the C-ABI of include/vdwlb.h)
  lattice       Plan / Lattice: one periodic D2Q9 or D1Q3 lattice on the GPU
  batch         Batch: many independent lattices in one persistent launch
  adjoint       VdwLBFunction: gradients through many steps (hand-written adjoint)
  phase         Appendix A phase diagrams over a grid of compositions
  verification  phase-diagram points run as lattice Boltzmann slabs
  inputs        seeded synthetic workloads (no lattice Boltzmann arithmetic)
  build         in-tree hipcc build of libvdwlb.so
"""
from . import inputs, vdwlb  # noqa: F401

__all__ = ["inputs", "vdwlb"]
