"""MI355X (gfx950) implementation of the matrix-free SIPG-DG Laplacian, its
vertex-patch multigrid preconditioner and the FGMRES Poisson solver of
Cui, "Acceleration of Tensor-Product Operations with Tensor Cores"
(arXiv 2407.09621).

The compute lives in the HIP library ``libsipg.so`` (C ABI: include/sipg.h);
``sipg`` is its ctypes binding.  Build with
``python -m paper_2407_09621_amd.build``.
"""
from .sipg import Batch, Network, Problem, SipgError, load_library, LIB_PATH  # noqa: F401
