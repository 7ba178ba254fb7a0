"""Differentiable expanded encoding (torch.autograd) on the HIP kernels.

* ``ExpEncForward``  y = A(k, dw0) x : backward = the adjoint kernel for x and
  the field-gradient kernel (``expenc_field_grad``) for k and dw0;
* ``ExpEncAdjoint``  x = A(k, dw0)^H y : backward = the forward kernel for y
  and the field-gradient kernel with the roles of the arguments swapped;
* ``WaveletFwd`` / ``WaveletInv`` : W and W^H (orthonormal, so each is the
  other's backward);
* ``SoftThreshold`` : the prox of the l1 term, backward = ``soft_threshold_vjp``;
* ``Axpby`` : a x + b y (real a, b) in the library (``expenc_axpby``), for
  the linear steps of an iteration: the residual, the gradient step and the
  momentum; its backward is the same call with the scalars;
* ``unrolled_fista`` : K iterations of FISTA on eq. 1 with fixed L and lambda,
  optionally with per-iteration checkpointing (each iteration is recomputed
  in the backward pass from its inputs instead of storing its intermediates).

Complex gradients follow torch's convention grad = dL/dRe + i dL/dIm.
Between the library calls only layout moves remain in torch (the crop of
the encoded block, its zero padding to the wavelet grid, reshapes).
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import torch
from torch.utils.checkpoint import checkpoint

from . import _binding as _b
from . import expenc as _e


class OperatorSpec:
    """The parts of an encoding operator that are not differentiated:
    grid, coil maps, sample times and the basis (maps, or the solid
    harmonics of a grid)."""

    def __init__(self, nx: int, ny: int, smaps: torch.Tensor, time: torch.Tensor,
                 basis: Optional[torch.Tensor] = None, sh_grid: Optional[Sequence[float]] = None):
        if basis is None and sh_grid is None:
            raise ValueError("give basis maps or sh_grid")
        self.nx, self.ny = nx, ny
        self.smaps, self.time, self.basis, self.sh_grid = smaps, time, basis, sh_grid

    def operator(self, coef: torch.Tensor, dw0: Optional[torch.Tensor]) -> _e.Operator:
        coef = coef.detach().contiguous()
        dw0 = None if dw0 is None else dw0.detach().contiguous()
        return _e.Operator(self.nx, self.ny, self.smaps, coef, self.time,
                           None if self.sh_grid is not None else self.basis, dw0, sh_grid=self.sh_grid,
                           nbasis=coef.shape[1])


def field_grad(op: _e.Operator, w: torch.Tensor, kk: torch.Tensor, want_coef=True, want_dw0=True):
    """grad_coef [T][L] and grad_dw0 [R] (float64) of the field-gradient kernel
    for one problem: w [R], kk [T][C] (see expenc_field_grad)."""
    w = w.reshape(op.npix).contiguous()
    kk = kk.reshape(op.nsamples, op.ncoils).contiguous()
    gc = torch.empty((op.nsamples, op.nbasis), dtype=torch.float64, device=op.device) if want_coef and op.nbasis \
        else None
    gd = torch.empty(op.npix, dtype=torch.float64, device=op.device) if want_dw0 else None
    ws = op.workspace(_b.WS_FIELD_GRAD, 1, _b.FP32)
    _b.check(_b.lib().expenc_field_grad(ctypes.byref(op._c), _b.FP32, _e._ptr(w), _e._ptr(kk), _e._ptr(gc),
                                        _e._ptr(gd), _e._ptr(ws), ws.numel(), _e._stream(op.device)),
             "expenc_field_grad")
    return gc, gd


def _field_grads(op, ws_batch, kks_batch, want_coef, want_dw0):
    gc_tot = gd_tot = None
    for w, kk in zip(ws_batch, kks_batch):
        gc, gd = field_grad(op, w, kk, want_coef, want_dw0)
        gc_tot = gc if gc_tot is None else gc_tot + gc
        gd_tot = gd if gd_tot is None else gd_tot + gd
    return gc_tot, gd_tot


class ExpEncForward(torch.autograd.Function):
    """y = A(coef, dw0) x ;  x [B][R] complex64 -> y [B][T][C]."""

    @staticmethod
    def forward(ctx, x, coef, dw0, spec: OperatorSpec):
        op = spec.operator(coef, dw0)
        y = _e.forward(x.contiguous(), op)
        ctx.spec = spec
        ctx.has_dw0 = dw0 is not None
        ctx.save_for_backward(x, coef, dw0 if dw0 is not None else coef.new_empty(0))
        return y

    @staticmethod
    def backward(ctx, g):
        x, coef, dw0 = ctx.saved_tensors
        dw0 = dw0 if ctx.has_dw0 else None
        op = ctx.spec.operator(coef, dw0)
        g = g.contiguous()
        gx = _e.adjoint(g, op).reshape(x.shape) if ctx.needs_input_grad[0] else None
        want_c, want_d = ctx.needs_input_grad[1], ctx.has_dw0 and ctx.needs_input_grad[2]
        gc = gd = None
        if want_c or want_d:
            xb = x.reshape(-1, op.npix)
            gb = g.reshape(-1, op.nsamples, op.ncoils)
            gc, gd = _field_grads(op, xb, gb, want_c, want_d)
        return gx, gc, gd, None


class ExpEncAdjoint(torch.autograd.Function):
    """x = A(coef, dw0)^H y ;  y [B][T][C] complex64 -> x [B][R]."""

    @staticmethod
    def forward(ctx, y, coef, dw0, spec: OperatorSpec):
        op = spec.operator(coef, dw0)
        x = _e.adjoint(y.contiguous(), op)
        ctx.spec = spec
        ctx.has_dw0 = dw0 is not None
        ctx.save_for_backward(y, coef, dw0 if dw0 is not None else coef.new_empty(0))
        return x

    @staticmethod
    def backward(ctx, gx):
        y, coef, dw0 = ctx.saved_tensors
        dw0 = dw0 if ctx.has_dw0 else None
        op = ctx.spec.operator(coef, dw0)
        gx = gx.contiguous()
        gy = _e.forward(gx, op).reshape(y.shape) if ctx.needs_input_grad[0] else None
        want_c, want_d = ctx.needs_input_grad[1], ctx.has_dw0 and ctx.needs_input_grad[2]
        gc = gd = None
        if want_c or want_d:
            gxb = gx.reshape(-1, op.npix)
            yb = y.reshape(-1, op.nsamples, op.ncoils)
            gc, gd = _field_grads(op, gxb, yb, want_c, want_d)
        return gy, gc, gd, None


class WaveletFwd(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, levels: int, wavelet: str):
        ctx.levels, ctx.wavelet = levels, wavelet
        return _e.wavelet_fwd(x.contiguous(), levels, wavelet)

    @staticmethod
    def backward(ctx, g):
        return _e.wavelet_inv(g.contiguous(), ctx.levels, ctx.wavelet), None, None


class WaveletInv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, levels: int, wavelet: str):
        ctx.levels, ctx.wavelet = levels, wavelet
        return _e.wavelet_inv(w.contiguous(), levels, wavelet)

    @staticmethod
    def backward(ctx, g):
        return _e.wavelet_fwd(g.contiguous(), ctx.levels, ctx.wavelet), None, None


class SoftThreshold(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, tau: float, levels: int):
        w = w.contiguous()
        ctx.tau, ctx.levels = float(tau), levels
        ctx.save_for_backward(w)
        return _e.soft_threshold(w, tau, levels)

    @staticmethod
    def backward(ctx, g):
        (w,) = ctx.saved_tensors
        wb = w.reshape((-1,) + tuple(w.shape[-2:]))
        g = g.contiguous().reshape(wb.shape)
        out = torch.empty_like(wb)
        _b.check(_b.lib().soft_threshold_vjp(wb.shape[2], wb.shape[1], ctx.levels, wb.shape[0], _e._ptr(wb),
                                             _e._ptr(g), _e._ptr(out), ctx.tau, _e._stream(w.device)),
                 "soft_threshold_vjp")
        return out.reshape(w.shape), None, None


class Axpby(torch.autograd.Function):
    """out = a x + b y for complex64 x, y of one shape and real a, b."""

    @staticmethod
    def forward(ctx, a: float, x, b: float, y):
        ctx.a, ctx.b = float(a), float(b)
        return _e.axpby(ctx.a, x.contiguous(), ctx.b, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        gx = _e.axpby(ctx.a, g, 0.0, g) if ctx.needs_input_grad[1] else None
        gy = _e.axpby(ctx.b, g, 0.0, g) if ctx.needs_input_grad[3] else None
        return None, gx, None, gy


def momentum(n_iter: int):
    """beta_k = (t_k - 1)/t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2."""
    out, t = [], 1.0
    for _ in range(n_iter):
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out.append((t - 1.0) / tn)
        t = tn
    return out


def _iteration(z, x_prev, y, coef, dw0, spec, L, lam, beta, levels, wavelet, nxp, nyp):
    nx, ny = spec.nx, spec.ny
    zc = z[..., :ny, :nx].reshape(z.shape[0], nx * ny).contiguous()
    r = Axpby.apply(1.0, ExpEncForward.apply(zc, coef, dw0, spec), -1.0, y)
    g = ExpEncAdjoint.apply(r, coef, dw0, spec).reshape(z.shape[0], ny, nx)
    g = torch.nn.functional.pad(torch.view_as_real(g), (0, 0, 0, nxp - nx, 0, nyp - ny))
    v = Axpby.apply(1.0, z, -2.0 / L, torch.view_as_complex(g.contiguous()))
    w = SoftThreshold.apply(WaveletFwd.apply(v, levels, wavelet), lam / L, levels)
    x = WaveletInv.apply(w, levels, wavelet)
    return x, Axpby.apply(1.0 + beta, x, -beta, x_prev)


def unrolled_fista(y, coef, dw0, spec: OperatorSpec, L: float, lam: float, n_iter: int, levels: int,
                   wavelet: str = "db4", nx_pad: int = 0, ny_pad: int = 0, use_checkpoint: bool = True):
    """x_hat = crop(x_K) of K FISTA iterations on eq. 1 (x_0 = z_1 = 0), as a
    differentiable function of y [B][T][C], coef [T][L] and dw0 [R]."""
    m = 1 << levels
    nxp = nx_pad or -(-spec.nx // m) * m
    nyp = ny_pad or -(-spec.ny // m) * m
    B = y.shape[0]
    x_prev = torch.zeros((B, nyp, nxp), dtype=torch.complex64, device=y.device)
    z = x_prev
    for beta in momentum(n_iter):
        args = (z, x_prev, y, coef, dw0, spec, L, lam, beta, levels, wavelet, nxp, nyp)
        if use_checkpoint:
            x, z = checkpoint(_iteration, *args, use_reentrant=False)
        else:
            x, z = _iteration(*args)
        x_prev = x
    return x_prev[..., :spec.ny, :spec.nx]
