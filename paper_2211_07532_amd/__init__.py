"""MI355X (gfx950) expanded-encoding compressed-sensing reconstruction.

The hot path of eq. 1 of Varela-Mattatall, Dubovan et al. -- repeated
application of the expanded encoding operator A_exp and its adjoint inside
FISTA, with a Haar/Daubechies wavelet prox -- as hand-written HIP kernels
behind a C ABI (include/expenc.h, libexpenc.so).  This package is the thin
Python binding; it loads the in-tree library and raises if it is missing.
"""
from .expenc import (Operator, sh_basis, forward, adjoint, lipschitz, wavelet_fwd, wavelet_inv,  # noqa: F401
                     wavelet_prox, soft_threshold, fista, fista_batched, cg, prewhiten, coil_compress, swt_fwd, swt_inv,
                     sigma_weights, fista_balanced, BalancedResult, FistaResult, axpby,
                     PRECISIONS, WAVELETS, ANCHORS)
from ._binding import lib, path as library_path, ExpencError, LibraryMissing  # noqa: F401
