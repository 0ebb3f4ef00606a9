"""MI355X-native FP64 selected inversion of band-plus-arrowhead SPD matrices.

Tile Cholesky A = L L^T on the band and arrow tiles, log det A, and the
two-phase backward recurrence that yields Sigma = A^{-1} on the tile pattern of
L (arXiv 2504.19171, Sec. III).  The compute runs in hand-written HIP kernels
for gfx950 behind the C ABI declared in ``include/stiles.h``; the Python module
:mod:`paper_2504_19171_amd.stiles` marshals arguments to it.
"""

__all__ = ["autotune", "grad", "inputs", "layout", "serve", "stiles"]
