"""Python binding of the expanded-encoding CS library (torch tensors in,
torch tensors out).  Each function marshals device pointers, sizes and the
current HIP stream into one C-ABI call of libexpenc.so; all arithmetic runs
in the library's HIP kernels.  Tensors must live on a ROCm device.

Layouts (see include/expenc.h): images [B][ny][nx] (or [B][R]) complex64,
k-space [B][T][C] complex64, field arrays float64.

Workspaces are allocated by the binding and kept for reuse, one per operator,
call kind and current stream (per device and stream for batched solves):
calls on one stream are ordered by it, calls on different streams get
different workspaces.  Several host threads that issue calls on ONE stream
with one operator must take turns, since their launches would interleave.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _binding as _b
from ._binding import FP32, BF16_SPLIT, FP16_SPLIT, HAAR, DB4, check

PRECISIONS = {"fp32": FP32, "bf16": BF16_SPLIT, "bf16_split": BF16_SPLIT, "fp16": FP16_SPLIT,
              "fp16_split": FP16_SPLIT}
WAVELETS = {"haar": HAAR, "db4": DB4}
# anchors of the split forms' gradient (see EXPENC_ANCHOR_* in include/expenc.h)
ANCHORS = {"split": _b.EXPENC_ANCHOR_SPLIT, "fp32": _b.EXPENC_ANCHOR_FP32, "ends": _b.EXPENC_ANCHOR_ENDS}


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _wav(w) -> int:
    return WAVELETS[w] if isinstance(w, str) else int(w)


def _anchor(a) -> int:
    return ANCHORS[a] if isinstance(a, str) else int(a)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _status(ws: torch.Tensor, where: str, raise_on_failure: bool) -> int:
    """Outcome flags of the call that used ws (expenc_solve_status; waits for the
    current stream).  Raises ExpencError on a failure if raise_on_failure."""
    st = _b.lib().expenc_solve_status(_ptr(ws), _stream(ws.device))
    if st in (_b.EXPENC_EINVAL, _b.EXPENC_EHIP) or (st != _b.EXPENC_OK and raise_on_failure):
        check(st, where)
    return st


def _need(t: torch.Tensor, dtype, name: str, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Operator:
    """One expanded-encoding operator: A[(t,c), r] = S_c(r) exp(i phi(t, r)),
    phi = sum_l coef[t, l] basis[l, r] + dw0[r] time[t].

    basis [L][R] f64, coef [T][L] f64 (rad per basis unit), time [T] f64 (s),
    dw0 [R] f64 (rad/s) or None, smaps [C][R] complex64; image nx x ny.
    With sh_grid=(fov_x, fov_y, z0) the basis is declared to be the real
    solid harmonics on that grid (basis may then be None); the library can
    then evaluate the phase in polynomial form."""

    def __init__(self, nx: int, ny: int, smaps, coef, time, basis, dw0=None, sh_grid=None, nbasis=None):
        dev = smaps.device
        self.device = dev
        self.smaps = _need(smaps, torch.complex64, "smaps", dev)
        self.time = _need(time, torch.float64, "time", dev)
        self.nx, self.ny = int(nx), int(ny)
        self.ncoils = smaps.shape[0]
        self.nsamples = time.shape[0]
        self.sh_grid = sh_grid
        if sh_grid is not None and basis is None and coef is not None and coef.numel() > 0:
            self.basis = None
            self.coef = _need(coef, torch.float64, "coef", dev)
            self.nbasis = coef.shape[1] if nbasis is None else int(nbasis)
            if coef.shape != (self.nsamples, self.nbasis):
                raise ValueError(f"coef must be [T][L] = [{self.nsamples}][{self.nbasis}]")
        elif basis is None or basis.numel() == 0:
            self.nbasis = 0
            self.basis = self.coef = None
        else:
            self.basis = _need(basis, torch.float64, "basis", dev)
            self.coef = _need(coef, torch.float64, "coef", dev)
            self.nbasis = basis.shape[0]
            if coef.shape != (self.nsamples, self.nbasis):
                raise ValueError(f"coef must be [T][L] = [{self.nsamples}][{self.nbasis}]")
            if basis.shape[1] != self.nx * self.ny:
                raise ValueError("basis must be [L][nx*ny]")
        self.dw0 = None if dw0 is None else _need(dw0, torch.float64, "dw0", dev)
        if smaps.shape[1] != self.nx * self.ny:
            raise ValueError("smaps must be [C][nx*ny]")
        self._c = _b.ExpencOp(self.nx, self.ny, self.ncoils, self.nbasis, self.nsamples,
                              None if self.basis is None else self.basis.data_ptr(),
                              None if self.coef is None else self.coef.data_ptr(),
                              self.time.data_ptr(),
                              None if self.dw0 is None else self.dw0.data_ptr(),
                              self.smaps.data_ptr(),
                              _b.BASIS_SH if sh_grid is not None else _b.BASIS_MAPS, 0,
                              *(tuple(float(v) for v in sh_grid) if sh_grid is not None else (0.0, 0.0, 0.0)))
        self._ws = {}

    @property
    def npix(self) -> int:
        return self.nx * self.ny

    def workspace(self, what: int, batch: int = 1, precision=FP32, nx_pad: int = 0, ny_pad: int = 0):
        n = _b.lib().expenc_workspace_size(ctypes.byref(self._c), batch, _prec(precision), what, nx_pad, ny_pad)
        if n == 0:
            raise _b.ExpencError(_b.EXPENC_EINVAL, "expenc_workspace_size")
        key = (what, batch, _prec(precision), nx_pad, ny_pad, _stream(self.device).value)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n:
            ws = torch.empty(n, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws


def sh_basis(nx: int, ny: int, fov_x: float, fov_y: float, z0: float, nbasis: int, device="cuda") -> torch.Tensor:
    """Real solid-harmonic field basis [L][R] (float64) on the pixel grid."""
    out = torch.empty((nbasis, nx * ny), dtype=torch.float64, device=device)
    check(_b.lib().expenc_sh_basis(nx, ny, fov_x, fov_y, z0, nbasis, _ptr(out) if nbasis else None,
                                   _stream(out.device)), "expenc_sh_basis")
    return out


def forward(x: torch.Tensor, op: Operator, precision="fp32", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x.  x: [R] or [B][R] (or [B][ny][nx]) complex64 -> y [B][T][C]."""
    single = x.dim() == 1
    xb = x.reshape(1 if single else x.shape[0], op.npix)
    _need(xb, torch.complex64, "x", op.device)
    batch = xb.shape[0]
    y = out if out is not None else torch.empty((batch, op.nsamples, op.ncoils), dtype=torch.complex64,
                                                device=op.device)
    _need(y, torch.complex64, "y", op.device)
    ws = op.workspace(_b.WS_FORWARD, batch, precision)
    check(_b.lib().expenc_forward(ctypes.byref(op._c), batch, _prec(precision), _ptr(xb), _ptr(y), _ptr(ws),
                                  ws.numel(), _stream(op.device)), "expenc_forward")
    return y[0] if single else y


def adjoint(y: torch.Tensor, op: Operator, precision="fp32", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A^H y.  y: [T][C] or [B][T][C] complex64 -> x [B][R]."""
    single = y.dim() == 2
    yb = y.reshape(1 if single else y.shape[0], op.nsamples, op.ncoils)
    _need(yb, torch.complex64, "y", op.device)
    batch = yb.shape[0]
    x = out if out is not None else torch.empty((batch, op.npix), dtype=torch.complex64, device=op.device)
    _need(x, torch.complex64, "x", op.device)
    ws = op.workspace(_b.WS_ADJOINT, batch, precision)
    check(_b.lib().expenc_adjoint(ctypes.byref(op._c), batch, _prec(precision), _ptr(yb), _ptr(x), _ptr(ws),
                                  ws.numel(), _stream(op.device)), "expenc_adjoint")
    return x[0] if single else x


def lipschitz(op: Operator, v0: torch.Tensor, n_iter: int, precision="fp32") -> torch.Tensor:
    """L = 2 lambda_max(A^H A) by power iteration from v0 [R]; a device float64 scalar."""
    _need(v0, torch.complex64, "v0", op.device)
    out = torch.empty(1, dtype=torch.float64, device=op.device)
    ws = op.workspace(_b.WS_LIPSCHITZ, 1, precision)
    check(_b.lib().expenc_lipschitz(ctypes.byref(op._c), _prec(precision), n_iter, _ptr(v0), _ptr(out), _ptr(ws),
                                    ws.numel(), _stream(op.device)), "expenc_lipschitz")
    return out


def wavelet_fwd(x: torch.Tensor, levels: int, wavelet="db4", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """W x for x [ny][nx] or [B][ny][nx] complex64 (Mallat layout)."""
    xb = x.reshape((-1,) + tuple(x.shape[-2:]))
    _need(xb, torch.complex64, "x", None)
    w = out if out is not None else torch.empty_like(xb)
    check(_b.lib().wavelet_fwd(xb.shape[2], xb.shape[1], levels, _wav(wavelet), xb.shape[0], _ptr(xb), _ptr(w),
                               _stream(x.device)), "wavelet_fwd")
    return w.reshape(x.shape)


def wavelet_inv(w: torch.Tensor, levels: int, wavelet="db4", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    wb = w.reshape((-1,) + tuple(w.shape[-2:]))
    _need(wb, torch.complex64, "w", None)
    x = out if out is not None else torch.empty_like(wb)
    check(_b.lib().wavelet_inv(wb.shape[2], wb.shape[1], levels, _wav(wavelet), wb.shape[0], _ptr(wb), _ptr(x),
                               _stream(w.device)), "wavelet_inv")
    return x.reshape(w.shape)


def soft_threshold(w: torch.Tensor, tau: float, levels: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    wb = w.reshape((-1,) + tuple(w.shape[-2:]))
    _need(wb, torch.complex64, "w", None)
    o = out if out is not None else torch.empty_like(wb)
    check(_b.lib().soft_threshold(wb.shape[2], wb.shape[1], levels, wb.shape[0], _ptr(wb), _ptr(o), float(tau),
                                  _stream(w.device)), "soft_threshold")
    return o.reshape(w.shape)


def wavelet_prox(v: torch.Tensor, levels: int, tau: torch.Tensor, x_prev: torch.Tensor, beta: float,
                 wavelet="db4", out=None):
    """One prox step with momentum: x = W^H S_tau(W v), z = x + beta (x - x_prev)
    for v, x_prev [B][ny][nx] complex64 and tau [B] float64 (device).  v is
    overwritten (the transform's scratch).  Returns (x, z, w); out may give
    preallocated (x, z, w)."""
    vb = v.reshape((-1,) + tuple(v.shape[-2:]))
    _need(vb, torch.complex64, "v", None)
    pb = x_prev.reshape(vb.shape)
    _need(pb, torch.complex64, "x_prev", v.device)
    _need(tau, torch.float64, "tau", v.device)
    if tau.numel() != vb.shape[0]:
        raise ValueError("tau needs one value per image")
    x, z, w = out if out is not None else (torch.empty_like(vb), torch.empty_like(vb), torch.empty_like(vb))
    check(_b.lib().wavelet_prox(vb.shape[2], vb.shape[1], levels, _wav(wavelet), vb.shape[0], _ptr(vb), _ptr(w),
                                _ptr(x), _ptr(pb), _ptr(z), float(beta), _ptr(tau), _stream(v.device)),
          "wavelet_prox")
    return x.reshape(v.shape), z.reshape(v.shape), w.reshape(v.shape)


def axpby(a: float, x: torch.Tensor, b: float, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """a x + b y for complex64 tensors of one shape (a, b real), in the library."""
    _need(x, torch.complex64, "x", None)
    _need(y, torch.complex64, "y", x.device)
    if x.shape != y.shape:
        raise ValueError("x and y must have one shape")
    o = out if out is not None else torch.empty_like(x)
    _need(o, torch.complex64, "out", x.device)
    check(_b.lib().expenc_axpby(x.numel(), float(a), _ptr(x), float(b), _ptr(y), _ptr(o), _stream(x.device)),
          "expenc_axpby")
    return o


@dataclasses.dataclass
class FistaResult:
    x: torch.Tensor                      # [B][ny][nx]
    lipschitz: float
    lam: list
    tau: list
    objective: Optional[torch.Tensor]    # [B][n_iter] float64
    status: Optional[int] = None         # expenc_solve_status (None when not read)


def fista(y: torch.Tensor, op: Operator, n_iter: int, levels: int, wavelet="db4", precision="fp32",
          lipschitz: float = 0.0, lam: float = -1.0, lambda_factor: float = 1e-3, power_v0=None,
          n_power: int = 30, nx_pad: int = 0, ny_pad: int = 0, ista: bool = False, refine_every: int = 0,
          trace: bool = False, sync_scalars: bool = True, check_status: bool = True, anchor="split"):
    """FISTA on eq. 1 (see fista_solve in include/expenc.h).  Returns a FistaResult.
    anchor: precision of the split forms' gradient anchors, "split" (every
    anchor after the first in the split form), "fp32" (every anchor in FP32)
    or "ends" (as "split" with the last one in FP32).
    With sync_scalars the call waits for the solve and reads its status word:
    a non-finite iterate (or, with trace=True, an objective above F(0))
    raises ExpencError when check_status, else is returned in .status."""
    single = y.dim() == 2
    yb = y.reshape(1 if single else y.shape[0], op.nsamples, op.ncoils)
    _need(yb, torch.complex64, "y", op.device)
    batch = yb.shape[0]
    m = 1 << levels
    nxp = nx_pad or -(-op.nx // m) * m
    nyp = ny_pad or -(-op.ny // m) * m
    x = torch.empty((batch, op.ny, op.nx), dtype=torch.complex64, device=op.device)
    obj = torch.empty((batch, max(n_iter, 1)), dtype=torch.float64, device=op.device) if trace else None
    sc = torch.zeros(2 + 2 * batch, dtype=torch.float64, device=op.device)
    if lipschitz <= 0 and power_v0 is None:
        raise ValueError("lipschitz <= 0 needs power_v0 (the seeded start vector)")
    opts = _b.FistaOpts(n_iter, _prec(precision), _wav(wavelet), levels, nxp, nyp, int(ista), refine_every,
                        n_power, 0, float(lipschitz), float(lam), float(lambda_factor),
                        None if power_v0 is None else _need(power_v0, torch.complex64, "power_v0",
                                                            op.device).data_ptr(),
                        None if obj is None else obj.data_ptr(), sc.data_ptr(), _anchor(anchor))
    ws = op.workspace(_b.WS_FISTA, batch, precision, nxp, nyp)
    check(_b.lib().fista_solve(ctypes.byref(op._c), batch, _ptr(yb), _ptr(x), ctypes.byref(opts), _ptr(ws),
                               ws.numel(), _stream(op.device)), "fista_solve")
    if sync_scalars:
        s = sc.cpu().tolist()
        st = _status(ws, "fista_solve", check_status)
        res = FistaResult(x[0] if single else x, s[0], s[2:2 + batch], s[2 + batch:2 + 2 * batch], obj, st)
    else:
        res = FistaResult(x[0] if single else x, float("nan"), [], [], obj)
    return res


def _coil_ws(ncoils: int, nsamples: int, device):
    n = _b.lib().expenc_coil_workspace_size(ncoils, nsamples)
    if n == 0:
        raise _b.ExpencError(_b.EXPENC_EINVAL, "expenc_coil_workspace_size")
    return torch.empty(n, dtype=torch.uint8, device=device)


def prewhiten(psi: torch.Tensor, y: Optional[torch.Tensor] = None, smaps: Optional[torch.Tensor] = None):
    """In place: every coil vector of y [..., C] and smaps [C, ...] becomes L^{-1} v with
    psi = L L^H (psi [C][C] complex128).  Returns (y, smaps)."""
    C = psi.shape[0]
    dev = psi.device
    _need(psi, torch.complex128, "psi", dev)
    ny = 0 if y is None else y.numel() // C
    npix = 0 if smaps is None else smaps.numel() // C
    if y is not None:
        _need(y, torch.complex64, "y", dev)
    if smaps is not None:
        _need(smaps, torch.complex64, "smaps", dev)
    ws = _coil_ws(C, 0, dev)
    check(_b.lib().expenc_prewhiten(C, _ptr(psi), ny, _ptr(y), npix, _ptr(smaps), _ptr(ws), ws.numel(),
                                    _stream(dev)), "expenc_prewhiten")
    _status(ws, "expenc_prewhiten (noise covariance not positive definite)", True)
    return y, smaps


def coil_compress(y: torch.Tensor, nvirtual: int, smaps: Optional[torch.Tensor] = None):
    """Virtual coils from the leading eigenvectors of Y^H Y (y [..., C]).
    Returns (y_v [..., nv], smaps_v [nv, ...] or None, eigenvalues [C], V [C][C])."""
    C = y.shape[-1]
    dev = y.device
    _need(y, torch.complex64, "y", dev)
    n = y.numel() // C
    yv = torch.empty(tuple(y.shape[:-1]) + (nvirtual,), dtype=torch.complex64, device=dev)
    npix = 0
    sv = None
    if smaps is not None:
        _need(smaps, torch.complex64, "smaps", dev)
        npix = smaps.numel() // C
        sv = torch.empty((nvirtual,) + tuple(smaps.shape[1:]), dtype=torch.complex64, device=dev)
    v = torch.empty((C, C), dtype=torch.complex128, device=dev)
    w = torch.empty(C, dtype=torch.float64, device=dev)
    ws = _coil_ws(C, n, dev)
    check(_b.lib().expenc_coil_compress(C, nvirtual, n, _ptr(y), npix, _ptr(smaps), _ptr(yv), _ptr(sv), _ptr(v),
                                        _ptr(w), _ptr(ws), ws.numel(), _stream(dev)), "expenc_coil_compress")
    _status(ws, "expenc_coil_compress", True)
    return yv, sv, w, v


def _swt_ws(nx, ny, levels, batch, device):
    n = _b.lib().expenc_swt_workspace_size(nx, ny, levels, batch)
    if n == 0:
        raise _b.ExpencError(_b.EXPENC_EINVAL, "expenc_swt_workspace_size")
    return torch.empty(n, dtype=torch.uint8, device=device)


def swt_fwd(x: torch.Tensor, levels: int, wavelet="db4") -> torch.Tensor:
    """Undecimated wavelet coefficients [..., 3J+1, ny, nx] of x [..., ny, nx] (complex64)."""
    xb = x.reshape((-1,) + tuple(x.shape[-2:]))
    _need(xb, torch.complex64, "x", x.device)
    B, ny, nx = xb.shape
    w = torch.empty((B, 3 * levels + 1, ny, nx), dtype=torch.complex64, device=x.device)
    ws = _swt_ws(nx, ny, levels, B, x.device)
    check(_b.lib().swt_fwd(nx, ny, levels, _wav(wavelet), B, _ptr(xb), _ptr(w), _ptr(ws), ws.numel(),
                           _stream(x.device)), "swt_fwd")
    return w.reshape(tuple(x.shape[:-2]) + tuple(w.shape[1:]))


def swt_inv(w: torch.Tensor, levels: int, wavelet="db4") -> torch.Tensor:
    """W^H: image [..., ny, nx] from coefficients [..., 3J+1, ny, nx]."""
    wb = w.reshape((-1,) + tuple(w.shape[-3:]))
    _need(wb, torch.complex64, "w", w.device)
    B, nb, ny, nx = wb.shape
    if nb != 3 * levels + 1:
        raise ValueError(f"expected {3 * levels + 1} bands, got {nb}")
    x = torch.empty((B, ny, nx), dtype=torch.complex64, device=w.device)
    ws = _swt_ws(nx, ny, levels, B, w.device)
    check(_b.lib().swt_inv(nx, ny, levels, _wav(wavelet), B, _ptr(wb), _ptr(x), _ptr(ws), ws.numel(),
                           _stream(w.device)), "swt_inv")
    return x.reshape(tuple(w.shape[:-3]) + (ny, nx))


def sigma_weights(w: torch.Tensor, levels: int, scale: float = 1.0, counts: bool = False):
    """Per-band weights [B][3J+1] (float64) by the sigma/2 rule from undecimated
    coefficients w [B][3J+1][ny][nx]; with counts=True also the histograms [B][J][256]."""
    wb = w.reshape((-1,) + tuple(w.shape[-3:]))
    _need(wb, torch.complex64, "w", w.device)
    B, nb, ny, nx = wb.shape
    lam = torch.empty((B, nb), dtype=torch.float64, device=w.device)
    cnt = torch.empty((B, levels, 256), dtype=torch.int32, device=w.device) if counts else None
    n = _b.lib().expenc_sigma_workspace_size(nx, ny, levels, B)
    ws = torch.empty(n, dtype=torch.uint8, device=w.device)
    check(_b.lib().expenc_sigma_weights(nx, ny, levels, B, _ptr(wb), float(scale), _ptr(lam), _ptr(cnt), _ptr(ws),
                                        ws.numel(), _stream(w.device)), "expenc_sigma_weights")
    return (lam, cnt) if counts else lam


@dataclasses.dataclass
class BalancedResult:
    x: torch.Tensor           # [B][ny][nx] (or [ny][nx])
    lipschitz_a: float        # L_A = 2 lambda_max(A^H A)
    kappa: float
    lam: torch.Tensor         # [B][3J+1]


def fista_balanced(y: torch.Tensor, op: Operator, n_iter: int, levels: int = 1, wavelet="db4", precision="fp32",
                   lipschitz: float = 0.0, kappa: float = -1.0, lam: Optional[torch.Tensor] = None,
                   lambda_scale: float = 1.0, power_v0=None, n_power: int = 30, ista: bool = False,
                   refine_every: int = 0, anchor="split") -> BalancedResult:
    """Balanced FISTA with the undecimated wavelet (see fista_balanced_solve in include/expenc.h)."""
    single = y.dim() == 2
    yb = y.reshape(1 if single else y.shape[0], op.nsamples, op.ncoils)
    _need(yb, torch.complex64, "y", op.device)
    B = yb.shape[0]
    nb = 3 * levels + 1
    if lipschitz <= 0 and power_v0 is None:
        raise ValueError("lipschitz <= 0 needs power_v0 (the seeded start vector)")
    x = torch.empty((B, op.ny, op.nx), dtype=torch.complex64, device=op.device)
    sc = torch.zeros(3 + 2 * B * nb, dtype=torch.float64, device=op.device)
    if lam is not None:
        lam = _need(lam.reshape(B, nb).contiguous(), torch.float64, "lam", op.device)
    opts = _b.BalancedOpts(n_iter, _prec(precision), _wav(wavelet), levels, refine_every, n_power, int(ista),
                           _anchor(anchor),
                           float(lipschitz), float(kappa), float(lambda_scale),
                           None if power_v0 is None else _need(power_v0, torch.complex64, "power_v0",
                                                               op.device).data_ptr(),
                           None if lam is None else lam.data_ptr(), sc.data_ptr())
    n = _b.lib().fista_balanced_workspace_size(ctypes.byref(op._c), B, ctypes.byref(opts))
    if n == 0:
        raise _b.ExpencError(_b.EXPENC_EINVAL, "fista_balanced_workspace_size")
    key = ("balanced", B, _prec(precision), levels, _stream(op.device).value)
    ws = op._ws.get(key)
    if ws is None or ws.numel() < n:
        ws = torch.empty(n, dtype=torch.uint8, device=op.device)
        op._ws[key] = ws
    check(_b.lib().fista_balanced_solve(ctypes.byref(op._c), B, _ptr(yb), _ptr(x), ctypes.byref(opts), _ptr(ws),
                                        ws.numel(), _stream(op.device)), "fista_balanced_solve")
    s = sc.cpu()
    _status(ws, "fista_balanced_solve", True)
    return BalancedResult(x[0] if single else x, float(s[0]), float(s[1]), s[3:3 + B * nb].reshape(B, nb))


_batch_ws = {}


def fista_batched(ys: Sequence[torch.Tensor], ops: Sequence[Operator], n_iter: int, levels: int, wavelet="db4",
                  precision="fp32", lipschitz: float = 0.0, lam: float = -1.0, lambda_factor: float = 1e-3,
                  power_v0=None, n_power: int = 30, ista: bool = False, refine_every: int = 0,
                  check_status: bool = False, launch: str = "forked", anchor="split"):
    """Independent FISTA solves of problems (ys[i], ops[i]) in one call (see
    fista_solve_batched in include/expenc.h).  Every ys[i] is [T_i][C_i] (or
    [B][T_i][C_i] with one B for all).  Returns the list of x_i.  With
    check_status the call waits for the solves and raises ExpencError if any
    iterate turned non-finite (otherwise it returns without waiting).
    launch: "forked" (each group's own launches on forked streams) or
    "grouped" (lock-step groups sharing one launch per split
    contraction; split precisions, solid-harmonic operators)."""
    launches = {"forked": _b.EXPENC_BATCH_FORKED, "grouped": _b.EXPENC_BATCH_GROUPED}
    if launch not in launches:
        raise ValueError(f"launch must be one of {sorted(launches)}")
    if len(ys) != len(ops) or not ops:
        raise ValueError("need one y per operator")
    dev = ops[0].device
    single = ys[0].dim() == 2
    batch = 1 if single else ys[0].shape[0]
    ybs, xs = [], []
    for y, op in zip(ys, ops):
        yb = y.reshape(batch, op.nsamples, op.ncoils)
        _need(yb, torch.complex64, "y", dev)
        ybs.append(yb)
        xs.append(torch.empty((batch, op.ny, op.nx), dtype=torch.complex64, device=dev))
    if lipschitz <= 0 and power_v0 is None:
        raise ValueError("lipschitz <= 0 needs power_v0 (the seeded start vector)")
    opts = _b.FistaOpts(n_iter, _prec(precision), _wav(wavelet), levels, 0, 0, int(ista), refine_every,
                        n_power, launches[launch], float(lipschitz), float(lam), float(lambda_factor),
                        None if power_v0 is None else _need(power_v0, torch.complex64, "power_v0", dev).data_ptr(),
                        None, None, _anchor(anchor))
    n = len(ops)
    carr = (_b.ExpencOp * n)(*[op._c for op in ops])
    yp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ybs])
    xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
    need = _b.lib().fista_batched_workspace_size(n, carr, batch, ctypes.byref(opts))
    if need == 0:
        raise _b.ExpencError(_b.EXPENC_EINVAL, "fista_batched_workspace_size")
    wkey = (dev, _stream(dev).value)
    ws = _batch_ws.get(wkey)
    if ws is None or ws.numel() < need:
        _batch_ws.pop(wkey, None)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        _batch_ws[wkey] = ws
    check(_b.lib().fista_solve_batched(n, carr, batch, yp, xp, ctypes.byref(opts), _ptr(ws), ws.numel(),
                                       _stream(dev)), "fista_solve_batched")
    if check_status:
        _status(ws, "fista_solve_batched", True)
    return [x[0] if single else x for x in xs]


def cg(y: torch.Tensor, op: Operator, n_iter: int, precision="fp32", check_status: bool = False) -> torch.Tensor:
    """Least squares by CG on A^H A x = A^H y from 0, n_iter iterations -> x [B][R].
    With check_status the call waits and raises ExpencError on a non-finite iterate."""
    single = y.dim() == 2
    yb = y.reshape(1 if single else y.shape[0], op.nsamples, op.ncoils)
    _need(yb, torch.complex64, "y", op.device)
    batch = yb.shape[0]
    x = torch.empty((batch, op.npix), dtype=torch.complex64, device=op.device)
    opts = _b.FistaOpts()
    opts.n_iter = n_iter
    opts.precision = _prec(precision)
    ws = op.workspace(_b.WS_CG, batch, precision)
    check(_b.lib().cg_solve(ctypes.byref(op._c), batch, _ptr(yb), _ptr(x), ctypes.byref(opts), _ptr(ws),
                            ws.numel(), _stream(op.device)), "cg_solve")
    if check_status:
        _status(ws, "cg_solve", True)
    return x[0] if single else x
