"""Reference gradients of an unrolled FISTA reconstruction (oracle, FP64).
Test infrastructure only.

The pipeline differentiated is the one used to learn through the CS
reconstruction (the paper names unrolled CS as future work, Discussion):

    y      = A(k, dw0) x_in                       (simulated k-space)
    x_hat  = FISTA_K(y; A(k, dw0), L, lambda)     (eq. 1, fixed L and lambda, x_0 = 0)
    loss   = ||x_hat - x_true||^2

and its gradient with respect to x_in, the field coefficients k_l(t) and
dw0(r).  Everything is written with plain PyTorch float64 CPU ops (the
encoding as exp of the phase times a matmul, the wavelet as its dense
per-level analysis matrices, the soft-threshold with torch.where) and
differentiated by torch's autograd.  It shares no code with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import wavelet as _wv


def _phase(coef, time, basis, dw0):
    ph = coef @ basis
    if dw0 is not None:
        ph = ph + time[:, None] * dw0[None, :]
    return ph


def forward(x, smaps, coef, time, basis, dw0):
    """y[t, c] = sum_r exp(i phi(t, r)) S_c(r) x(r)  (x: [R] complex128)."""
    e = torch.exp(1j * _phase(coef, time, basis, dw0))
    return e @ (smaps * x[None, :]).T


def adjoint(y, smaps, coef, time, basis, dw0):
    e = torch.exp(1j * _phase(coef, time, basis, dw0))
    return torch.sum(smaps.conj().T * (e.conj().T @ y), dim=1)


def _mats(n, levels, name):
    h = _wv.filters(name)
    return [torch.from_numpy(_wv.analysis_matrix(n >> j, h)).to(torch.complex128) for j in range(levels)]


def dwt2(x, mats):
    out = x
    for j, m in enumerate(mats):
        k = m.shape[0]
        blk = out[:k, :k]
        blk = m @ (blk @ m.T)              # rows, then columns
        out = out.clone()
        out[:k, :k] = blk
    return out


def idwt2(w, mats):
    out = w
    for m in reversed(mats):
        k = m.shape[0]
        blk = out[:k, :k]
        blk = m.T @ (blk @ m)
        out = out.clone()
        out[:k, :k] = blk
    return out


def soft(w, tau, levels):
    n = w.shape[-1]
    k = n >> levels
    mag = torch.abs(w)
    scale = torch.where(mag > tau, 1.0 - tau / torch.where(mag > 0, mag, torch.ones_like(mag)),
                        torch.zeros_like(mag))
    out = w * scale
    mask = torch.zeros_like(mag, dtype=torch.bool)
    mask[:k, :k] = True
    return torch.where(mask, w, out)


def fista(y, smaps, coef, time, basis, dw0, L, lam, n_iter, levels, name, n, n_pad):
    mats = _mats(n_pad, levels, name)
    x_prev = torch.zeros((n_pad, n_pad), dtype=torch.complex128)
    z = x_prev
    t = 1.0
    for _ in range(n_iter):
        zc = z[:n, :n].reshape(-1)
        g = adjoint(forward(zc, smaps, coef, time, basis, dw0) - y, smaps, coef, time, basis, dw0)
        gp = torch.zeros((n_pad, n_pad), dtype=torch.complex128)
        gp = gp.index_put((torch.arange(n)[:, None], torch.arange(n)[None, :]), g.reshape(n, n))
        v = z - (2.0 / L) * gp
        x = idwt2(soft(dwt2(v, mats), lam / L, levels), mats)
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x + ((t - 1.0) / tn) * (x - x_prev)
        x_prev = x
        t = tn
    return x_prev[:n, :n].reshape(-1)


def loss_and_grads(x_in, x_true, smaps, coef, time, basis, dw0, L, lam, n_iter, levels, name, n, n_pad):
    """(loss, d/dx_in [R] complex, d/dcoef [T][L], d/ddw0 [R]) in FP64;
    complex gradient in the convention dL/dRe + i dL/dIm."""
    t = lambda a: torch.from_numpy(np.asarray(a))
    xi = t(x_in).to(torch.complex128).requires_grad_(True)
    cf = t(coef).to(torch.float64).requires_grad_(True)
    dw = t(dw0).to(torch.float64).requires_grad_(True)
    sm, tm, bs = t(smaps).to(torch.complex128), t(time).to(torch.float64), t(basis).to(torch.float64)
    y = forward(xi, sm, cf, tm, bs, dw)
    xh = fista(y, sm, cf, tm, bs, dw, L, lam, n_iter, levels, name, n, n_pad)
    loss = torch.sum(torch.abs(xh - t(x_true).to(torch.complex128)) ** 2)
    loss.backward()
    # torch's complex gradient is the conjugate Wirtinger derivative times 2 for
    # real losses, i.e. dL/dRe + i dL/dIm
    return float(loss), xi.grad.numpy(), cf.grad.numpy(), dw.grad.numpy()
