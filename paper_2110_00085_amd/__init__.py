"""MI355X (gfx950) path-recycling scattering tomography.

Hot path of Czerninski & Schechner, arXiv 2110.00085: Monte-Carlo path
sampling through a voxel grid, recycled rendering with local estimation, the
loss gradient through the tomography path score function, and the
correction-factor statistics, all in hand-written HIP kernels behind the C
ABI of include/prt.h.  ``prt`` is the thin ctypes binding; ``api`` adds
owning handles and the torch autograd.Function.
"""
from . import prt  # noqa: F401

__all__ = ["prt"]
