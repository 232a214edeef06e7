"""MI355X (gfx950) hot path of extended diffraction tomography.

The method (Schlottmann, "Extended diffraction tomography", Section 2) splits
linear Born inversion over a depth-dependent reference into independent 1D
depth problems, one per midpoint wavenumber.  ``libedt.so`` (HIP, built by
``paper_0905_0238_amd.build``) computes the reference Green's tables, the
Gram matrices of the Born rows on MFMA, the damped Cholesky solves with FP64
refinement and the adjoint; this package only marshals torch tensors into its
C-ABI (``include/edt.h``).
"""
from . import _lib
from .edt import Plan, solve, pair_rows
from .pipeline import Pipeline
from .stream import Stream, cut_batches
from .autograd import EDTSolve, edt_solve

__all__ = ["Plan", "solve", "pair_rows", "Pipeline", "Stream", "cut_batches", "EDTSolve", "edt_solve", "_lib"]
