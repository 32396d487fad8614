"""Adaptive-multigrid Wilson-Dirac solver for AMD Instinct MI355X (gfx950).

Implements the hot path of Clark et al., "The removal of critical slowing
down" (Lattice 2008): the Wilson-Dirac stencil, chirality-split block
prolongation/restriction, the Galerkin coarse operator and the MR smoother
inside an MG-preconditioned flexible GCR solve.  The compute path is the C-ABI
library ``libwdmg.so`` (hand-written HIP kernels); ``wdmg`` is its Python
binding.  Import the binding explicitly: ``from paper_0811_4331_amd import wdmg``.
"""
