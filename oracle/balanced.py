"""The paper's own regulariser (oracle, FP64).  Test infrastructure only.

Methods 2.1 uses the undecimated wavelet transform with one level, a
regularisation weight per wavelet level set to sigma/2, where sigma is the
maximum of the histogram of the level's high-pass coefficient magnitudes of
W A^H y (a Rayleigh mode: the noise level), with weight 0 for the low-pass
band (Supporting Information S1), and solves the problem with balanced FISTA
(Methods 2.1, refs. 17 and 20).

* Undecimated (stationary, "a trous") periodised separable 2D transform with
  J levels on an N x N image (any N): at level j (step d = 2^j) the 1D
  filters act with taps spaced by d and scaled by 1/sqrt(2):
      lo(u)[i] = 2^-1/2 sum_k h[k] u[(i + d k) mod N],  hi: g instead of h,
  applied along x (the fast axis) and y.  Bands of level j, index 3j + b:
  b = 0 high x / low y, b = 1 low x / high y, b = 2 high / high; the last
  band (index 3J) is the coarsest low-pass; the next level transforms the
  low / low output.  With orthonormal filters this is a tight frame:
  W^H W = I, ||W x|| = ||x||.
* Weights: for each level, sigma = centre of the fullest of 256 equal bins
  over [0, 4 mean|w|) of the magnitudes of that level's three high-pass
  bands (values beyond the range are not counted; the lowest bin wins a
  tie); lambda = sigma / 2; the low-pass band is not penalised.
* Balanced model on the coefficients alpha (eq. 1's data term, no 1/2):
      F(alpha) = ||A W^H alpha - y||^2 + kappa/2 ||(I - W W^H) alpha||^2
                 + sum_b lambda_b ||alpha_b||_1
  solved by FISTA from alpha = 0 with step 1/L, L = 2 lambda_max(A^H A) +
  kappa, whose gradient is
      2 W A^H (A W^H beta - y) + kappa (beta - W W^H beta);
  the output is x = W^H alpha_K.  kappa -> infinity keeps alpha in the range
  of W (the analysis model of eq. 1); kappa = 0 is the synthesis model.
"""
from __future__ import annotations

import numpy as np

from . import wavelet as _wv


def _filt(u, f, d, axis):
    """2^-1/2 sum_k f[k] u[(i + d k) mod N] along axis."""
    out = np.zeros_like(u)
    for k, fk in enumerate(f):
        out = out + fk * np.roll(u, -d * k, axis=axis)
    return out / np.sqrt(2.0)


def _filt_adj(v, f, d, axis):
    """Adjoint of _filt: 2^-1/2 sum_k f[k] v[(i - d k) mod N]."""
    out = np.zeros_like(v)
    for k, fk in enumerate(f):
        out = out + fk * np.roll(v, d * k, axis=axis)
    return out / np.sqrt(2.0)


def swt2(x, levels: int, name: str):
    """[3J+1][N][N] coefficients of the N x N image x (x along axis 1)."""
    h = _wv.filters(name)
    g = _wv.highpass(h)
    u = np.asarray(x, dtype=np.complex128)
    bands = []
    for j in range(levels):
        d = 1 << j
        lx, hx = _filt(u, h, d, 1), _filt(u, g, d, 1)
        bands += [_filt(hx, h, d, 0), _filt(lx, g, d, 0), _filt(hx, g, d, 0)]
        u = _filt(lx, h, d, 0)
    bands.append(u)
    return np.stack(bands)


def iswt2(w, levels: int, name: str):
    """W^H: the adjoint of swt2 (its left inverse)."""
    h = _wv.filters(name)
    g = _wv.highpass(h)
    w = np.asarray(w, dtype=np.complex128)
    u = w[3 * levels]
    for j in reversed(range(levels)):
        d = 1 << j
        lx = _filt_adj(u, h, d, 0) + _filt_adj(w[3 * j + 1], g, d, 0)
        hx = _filt_adj(w[3 * j], h, d, 0) + _filt_adj(w[3 * j + 2], g, d, 0)
        u = _filt_adj(lx, h, d, 1) + _filt_adj(hx, g, d, 1)
    return u


def histogram_mode(mags, nbins: int = 256) -> float:
    """Centre of the fullest of nbins equal bins over [0, 4 mean)."""
    mags = np.asarray(mags, dtype=np.float64).ravel()
    top = 4.0 * np.mean(mags)
    if not top > 0:
        return 0.0
    width = top / nbins
    idx = np.floor(mags / width).astype(np.int64)
    counts = np.bincount(idx[idx < nbins], minlength=nbins)
    return (int(np.argmax(counts)) + 0.5) * width


def sigma_weights(w, levels: int, nbins: int = 256):
    """lambda per band ([3J+1]; 0 for the low-pass band) from the
    coefficients w = W A^H y: sigma/2 per level."""
    lam = np.zeros(3 * levels + 1)
    for j in range(levels):
        sigma = histogram_mode(np.abs(w[3 * j:3 * j + 3]), nbins)
        lam[3 * j:3 * j + 3] = sigma / 2.0
    return lam


def soft_bands(w, tau):
    """Per-band complex soft-threshold with thresholds tau[band] (0 = none)."""
    out = np.array(w, dtype=np.complex128)
    for b, t in enumerate(tau):
        if t > 0:
            m = np.abs(out[b])
            out[b] = out[b] * np.where(m > t, 1.0 - t / np.where(m > 0, m, 1.0), 0.0)
    return out


def objective(op, y, alpha, lam, kappa, levels, name):
    """F(alpha) of the balanced model (FP64)."""
    n = op.n
    x = iswt2(alpha, levels, name)
    r = op.A(x.reshape(-1)) - y
    p = alpha - swt2(x, levels, name)
    l1 = sum(lam[b] * np.sum(np.abs(alpha[b])) for b in range(len(lam)))
    assert x.shape == (n, n)
    return float(np.vdot(r, r).real + 0.5 * kappa * np.vdot(p, p).real + l1)


def fista(op, y, L_A: float, kappa: float, lam, n_iter: int, levels: int, name: str, ista: bool = False,
          trace: bool = False):
    """Balanced FISTA; returns x = W^H alpha_K ([N][N]) (and F per iteration)."""
    n = op.n
    L = L_A + kappa
    tau = np.asarray(lam, dtype=np.float64) / L
    alpha_prev = np.zeros((3 * levels + 1, n, n), dtype=np.complex128)
    beta = alpha_prev.copy()
    t = 1.0
    f = []
    for _ in range(n_iter):
        xb = iswt2(beta, levels, name)
        r = op.AH(op.A(xb.reshape(-1)) - y).reshape(n, n)
        grad = 2.0 * swt2(r, levels, name) + kappa * (beta - swt2(xb, levels, name))
        alpha = soft_bands(beta - grad / L, tau)
        tn = 1.0 if ista else (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = alpha + ((t - 1.0) / tn) * (alpha - alpha_prev)
        alpha_prev = alpha
        t = tn
        if trace:
            f.append(objective(op, y, alpha, lam, kappa, levels, name))
    x = iswt2(alpha_prev, levels, name)
    return (x, np.array(f)) if trace else x
