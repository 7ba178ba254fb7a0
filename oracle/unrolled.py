"""Reference gradients of an unrolled FISTA reconstruction (oracle, FP64).
Test infrastructure only.

The pipeline differentiated is the one used to learn through the CS
reconstruction (the paper names unrolled CS as future work, Discussion):

    y      = A(k, dw0) x_in                       (simulated k-space)
    x_hat  = FISTA_K(y; A(k, dw0), L, lambda)     (eq. 1, fixed L and lambda, x_0 = 0)
    loss   = ||x_hat - x_true||^2

and its gradient with respect to x_in, the field coefficients k_l(t) and
dw0(r).  Two derivations of the same gradient:

* ``loss_and_grads``: plain PyTorch float64 CPU ops (the encoding as exp of
  the phase times a matmul, the wavelet as its dense per-level analysis
  matrices, the soft-threshold with torch.where), differentiated by torch's
  autograd; it forms E whole, so it serves small sizes;
* ``reverse_loss_and_grads``: a hand-written reverse pass in NumPy FP64 over
  the blocked operators and field VJPs of ``encoding`` (never forming E
  whole), for the full differentiation workload.

Neither shares code with the GPU path.
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


# ---------------------------------------------------------------------------
# The same loss and gradients by a hand-written reverse pass in NumPy FP64
# over the blocked operators (encoding.forward / adjoint and the blocked
# field VJPs), which never form E whole, so it reaches the differentiation
# workload's size (128 x 128, 16 coils, 12000 samples).
# ---------------------------------------------------------------------------

def soft_vjp(u, gbar, tau, levels):
    """Vector-Jacobian product of the soft-threshold w -> w max(0, 1 - tau/|w|)
    at u (a.e. derivative, convention dL/dRe + i dL/dIm).  For |u| > tau the
    real-linear derivative is dw -> a dw + b n Re(conj(n) dw) with n = u/|u|,
    a = 1 - tau/|u|, b = tau/|u|; it is symmetric, so the VJP applies the
    same map to gbar.  Zero where |u| <= tau; identity on the coarsest LL."""
    mag = np.abs(u)
    live = mag > tau
    safe = np.where(live, mag, 1.0)
    nrm = np.where(live, u / safe, 0.0)
    a = np.where(live, 1.0 - tau / safe, 0.0)
    b = np.where(live, tau / safe, 0.0)
    out = a * gbar + b * nrm * np.real(np.conj(nrm) * gbar)
    k = u.shape[-1] >> levels
    m = u.shape[-2] >> levels
    out[..., :m, :k] = gbar[..., :m, :k]
    return out


def reverse_loss_and_grads(x_in, x_true, smaps, coef, time, basis, dw0, L, lam, n_iter, levels, name, n, n_pad):
    """Same outputs as loss_and_grads: (loss, d/dx_in [R] complex, d/dcoef [T][L],
    d/ddw0 [R]), complex gradients as dL/dRe + i dL/dIm.

    Forward pass (eq. 1 by FISTA, x_0 = z_1 = 0, fixed L and lambda, beta_k
    the FISTA momentum coefficients):
        y = A x_in;  r_k = A crop(z_k) - y;  g_k = A^H r_k;
        v_k = z_k - (2/L) pad(g_k);  u_k = W v_k;  x_k = W^H S_tau(u_k);
        z_{k+1} = x_k + beta_k (x_k - x_{k-1});  loss = ||crop(x_K) - x_true||^2.
    Reverse pass: each step's adjoint in the opposite order (W^H <-> W,
    pad <-> crop, A <-> A^H, the soft-threshold's VJP), with the field
    gradients of every A and A^H in the chain summed."""
    from . import encoding as enc
    from . import solve as slv
    from . import wavelet as wv

    def A(v):
        return enc.forward(v, smaps, coef, time, basis, dw0)

    def AH(v):
        return enc.adjoint(v, smaps, coef, time, basis, dw0)

    def pad(v):
        return slv.pad(v, n, n_pad)

    def crop(v):
        return slv.crop(v, n)

    x_in = np.asarray(x_in, dtype=np.complex128)
    tau = lam / L
    beta = slv.momentum_coeffs(n_iter)
    y = A(x_in)
    xs = [np.zeros((n_pad, n_pad), dtype=np.complex128)]
    z = xs[0]
    zcs, rs, us = [], [], []
    for k in range(n_iter):
        zc = crop(z)
        r = A(zc) - y
        v = z - (2.0 / L) * pad(AH(r))
        u = wv.dwt2(v, levels, name)
        x = wv.idwt2(wv.soft_threshold(u, tau, levels), levels, name)
        z = x + beta[k] * (x - xs[-1])
        zcs.append(zc)
        rs.append(r)
        us.append(u)
        xs.append(x)
    d = crop(xs[-1]) - np.asarray(x_true, dtype=np.complex128)
    loss = float(np.sum(np.abs(d) ** 2))

    xbar = [np.zeros_like(xs[0]) for _ in xs]
    xbar[-1] = pad(2.0 * d)
    zbar_next = np.zeros_like(xs[0])
    ybar = np.zeros_like(y)
    gcoef = np.zeros(coef.shape)
    gdw0 = np.zeros(smaps.shape[1]) if dw0 is not None else None

    def add_field(gc, gd):
        nonlocal gcoef
        gcoef = gcoef + gc
        if gdw0 is not None:
            gdw0[:] += gd

    for k in range(n_iter - 1, -1, -1):
        # z_{k+1} = (1 + beta_k) x_k - beta_k x_{k-1}
        xbar[k + 1] = xbar[k + 1] + (1.0 + beta[k]) * zbar_next
        xbar[k] = xbar[k] - beta[k] * zbar_next
        # x_k = W^H S_tau(u_k), u_k = W v_k
        vbar = wv.idwt2(soft_vjp(us[k], wv.dwt2(xbar[k + 1], levels, name), tau, levels), levels, name)
        # v_k = z_k - (2/L) pad(g_k)
        zbar = vbar.copy()
        gbar = -(2.0 / L) * crop(vbar)
        # g_k = A^H r_k
        rbar = A(gbar)
        add_field(*enc.field_vjp_adjoint(rs[k], gbar, smaps, coef, time, basis, dw0))
        # r_k = A crop(z_k) - y
        zbar = zbar + pad(AH(rbar))
        ybar = ybar - rbar
        add_field(*enc.field_vjp_forward(zcs[k], rbar, smaps, coef, time, basis, dw0))
        zbar_next = zbar
    # y = A x_in
    gx = AH(ybar)
    add_field(*enc.field_vjp_forward(x_in, ybar, smaps, coef, time, basis, dw0))
    return loss, gx, gcoef, gdw0
