"""Coil pre-whitening and coil compression (oracle, FP64).  Test
infrastructure only: imported by tests and by nothing in the library.

Methods 2.2.1: the k-space data were compressed to virtual coils to speed up
the reconstruction, and the noise correlation between receivers was removed
by pre-whitening before reconstruction.

* Pre-whitening: with the receivers' noise covariance Psi = L L^H (Cholesky,
  L lower triangular), data and coil maps become L^{-1} y and L^{-1} S (per
  sample / per pixel, over the coil index); the model y = A x keeps its form
  with the whitened maps, and the noise L^{-1} n is white.
* Compression: the virtual coils are the leading eigenvectors of the coil
  Gram matrix G = Y^H Y of the data Y [T][C] (equivalently its leading right
  singular vectors); with V_k = the first k of them (eigenvalues descending),
  y_v = Y V_k and the virtual maps S_v[j](r) = sum_c V_k[c, j] S_c(r), so the
  compressed data follow the same model with the virtual maps.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def prewhiten(psi, y, smaps):
    """(y_w [T][C], smaps_w [C][R]) = (L^{-1} y per sample, L^{-1} S per pixel)."""
    L = np.linalg.cholesky(np.asarray(psi, dtype=np.complex128))
    yw = scipy.linalg.solve_triangular(L, np.asarray(y, dtype=np.complex128).T, lower=True).T
    sw = scipy.linalg.solve_triangular(L, np.asarray(smaps, dtype=np.complex128), lower=True)
    return yw, sw


def gram(y):
    """G[a, b] = sum_t conj(y[t, a]) y[t, b]."""
    y = np.asarray(y, dtype=np.complex128)
    return y.conj().T @ y


def compression_matrix(y):
    """(eigenvalues descending [C], V [C][C] whose columns are the eigenvectors)."""
    w, v = np.linalg.eigh(gram(y))
    order = np.argsort(w)[::-1]
    return w[order], v[:, order]


def compress(y, smaps, nv):
    """(y_v [T][nv], smaps_v [nv][R], eigenvalues [C], V_k [C][nv])."""
    w, v = compression_matrix(y)
    vk = v[:, :nv]
    yv = np.asarray(y, dtype=np.complex128) @ vk
    sv = vk.T @ np.asarray(smaps, dtype=np.complex128)
    return yv, sv, w, vk
