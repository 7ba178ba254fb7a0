"""Wavelet transform W and the soft-threshold prox (oracle, FP64).
Test infrastructure only.

Eq. 1 penalises lambda * ||W x||_1 with W a wavelet transform (Methods 2.1
uses an undecimated transform; this build uses the decimated, periodised,
orthonormal separable 2D transform, for which the proximal step of the
l1 term is exact).  Filters:

* Haar: h = [1, 1] / sqrt(2);
* Daubechies with 4 vanishing moments (8 taps, "db4"), derived here by
  spectral factorisation of the Daubechies polynomial
  P(y) = sum_{k<4} C(3+k, k) y^k with |m0(w)|^2 = cos^8(w/2) P(sin^2(w/2)),
  keeping the extremal-phase factor: H(z) = sum_n h[n] z^-n has all of its
  zeros other than z = -1 strictly inside the unit circle.

One analysis level on a length-n vector v (n even, periodic):
    a[m] = sum_k h[k] v[(2m + k) mod n],  d[m] = sum_k g[k] v[(2m + k) mod n],
    g[k] = (-1)^k h[M-1-k].
2D: at each level, rows first then columns, on the current top-left
low-pass block; the output uses the Mallat layout [[LL, HL], [LH, HH]]
with the coarsest LL block at the top-left.  The inverse is the exact
adjoint (transpose) of the analysis.
"""
from __future__ import annotations

import math

import numpy as np


def haar_filter() -> np.ndarray:
    return np.array([1.0, 1.0]) / math.sqrt(2.0)


def daubechies_filter(p: int = 4) -> np.ndarray:
    """Extremal-phase Daubechies low-pass analysis filter with p vanishing
    moments (2p taps), normalised to sum(h) = sqrt(2)."""
    # Daubechies polynomial in y = sin^2(w/2)
    pc = [math.comb(p - 1 + k, k) for k in range(p)]          # ascending powers
    yroots = np.roots(pc[::-1]) if p > 1 else np.array([])
    # y = (2 - z - 1/z)/4  <=>  z^2 - (2 - 4y) z + 1 = 0 ; keep |z| < 1
    zr = []
    for yk in yroots:
        b = 2.0 - 4.0 * yk
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zr.append(z1 if abs(z1) < 1.0 else z2)
    # m0(z) ∝ (1 + z)^p * prod (z - z_k) as a polynomial in z (descending)
    poly = np.array([1.0 + 0j])
    for _ in range(p):
        poly = np.convolve(poly, [1.0, 1.0])
    for zk in zr:
        poly = np.convolve(poly, [1.0, -zk])
    c = np.real(poly)                      # descending powers of z
    # As H(z) = sum h[n] z^-n, the descending-power coefficients of a
    # polynomial with roots z_k give a filter whose zeros are exactly z_k.
    h = c / c.sum() * math.sqrt(2.0)
    return h


def filters(name: str) -> np.ndarray:
    if name == "haar":
        return haar_filter()
    if name == "db4":
        return daubechies_filter(4)
    raise ValueError(name)


def highpass(h: np.ndarray) -> np.ndarray:
    m = len(h)
    return np.array([(-1) ** k * h[m - 1 - k] for k in range(m)])


def analysis_matrix(n: int, h: np.ndarray) -> np.ndarray:
    """Dense n x n one-level periodised analysis matrix: rows 0..n/2-1 give
    the approximation a, rows n/2.. the detail d."""
    g = highpass(h)
    w = np.zeros((n, n))
    for m in range(n // 2):
        for k in range(len(h)):
            w[m, (2 * m + k) % n] += h[k]
            w[n // 2 + m, (2 * m + k) % n] += g[k]
    return w


def dwt2(x: np.ndarray, levels: int, name: str) -> np.ndarray:
    """Forward 2D transform of x [ny][nx] (or [B][ny][nx]), Mallat layout."""
    h = filters(name)
    out = np.array(x, dtype=np.complex128, copy=True)
    ny, nx = out.shape[-2:]
    if ny % (1 << levels) or nx % (1 << levels):
        raise ValueError("image sides must be multiples of 2^levels")
    for j in range(levels):
        my, mx = ny >> j, nx >> j
        wx = analysis_matrix(mx, h)
        wy = analysis_matrix(my, h)
        blk = out[..., :my, :mx]
        blk = blk @ wx.T                      # rows
        blk = np.swapaxes(np.swapaxes(blk, -1, -2) @ wy.T, -1, -2)   # columns
        out[..., :my, :mx] = blk
    return out


def idwt2(w: np.ndarray, levels: int, name: str) -> np.ndarray:
    """Inverse (adjoint) of dwt2."""
    h = filters(name)
    out = np.array(w, dtype=np.complex128, copy=True)
    ny, nx = out.shape[-2:]
    for j in reversed(range(levels)):
        my, mx = ny >> j, nx >> j
        wx = analysis_matrix(mx, h)
        wy = analysis_matrix(my, h)
        blk = out[..., :my, :mx]
        blk = np.swapaxes(np.swapaxes(blk, -1, -2) @ wy, -1, -2)     # columns
        blk = blk @ wx                                               # rows
        out[..., :my, :mx] = blk
    return out


def detail_mask(ny: int, nx: int, levels: int) -> np.ndarray:
    """True on every detail coefficient, False on the coarsest LL block
    (the low-pass band carries no penalty)."""
    m = np.ones((ny, nx), dtype=bool)
    m[: ny >> levels, : nx >> levels] = False
    return m


def soft_threshold(w: np.ndarray, tau: float, levels: int) -> np.ndarray:
    """Prox of tau * sum_detail |w_i| (complex modulus): each detail
    coefficient becomes w * max(0, 1 - tau/|w|) (0 when |w| <= tau); the
    coarsest LL block passes through unchanged."""
    w = np.asarray(w, dtype=np.complex128)
    ny, nx = w.shape[-2:]
    mag = np.abs(w)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    out = w * scale
    ll = ~detail_mask(ny, nx, levels)
    out[..., ll] = w[..., ll]
    return out
