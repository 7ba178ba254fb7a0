"""Solvers for eq. 1 and their helpers (oracle, FP64).  Test infrastructure only.

* ``fista``  -- FISTA (Beck-Teboulle) on eq. 1 exactly as written, i.e.
  f(x) = ||A crop(x) - y||^2 with no 1/2, so grad f = 2 pad(A^H(A crop(x) - y)),
  step 1/L, threshold tau = lambda/L (Methods 2.1: the paper's CS solver is
  FISTA, run for a fixed number of iterations).  With an orthonormal W the
  analysis, synthesis and balanced formulations coincide, so each
  iteration is  x_k = W^H S_tau(W(z_k - grad f(z_k)/L)),
  t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,  z_{k+1} = x_k + (t_k - 1)/t_{k+1} (x_k - x_{k-1}),
  starting from x_0 = z_1 = 0, t_1 = 1.  ``ista=True`` keeps t_k = 1.
* ``objective`` -- F(x) = ||A crop(x) - y||^2 + lambda * sum_detail |(W x)_i| (eq. 1).
* ``power_lipschitz`` -- L = 2 lambda_max(A^H A) by power iteration from a
  given start vector, Rayleigh quotient at the end.
* ``lambda_rule`` -- lambda from the zero-filled reconstruction (Methods
  2.1 derives lambda from W A^T y): here 1e-3 * max_r |(A^H y)(r)|.
* ``cg_ls`` -- conjugate gradient on the normal equations A^H A x = A^H y
  with early stopping after a fixed iteration count (Methods 2.1: 20).
* ``nrmse`` -- ||a - ref|| / ||ref|| (Methods 2.2.2 uses NRMSE to score
  reconstructions; the paper does not spell out the normalisation).

The image lives on an N_w x N_w wavelet grid (N_w = N rounded up to a
multiple of 2^J); the encoding sees only the top-left N x N crop.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import encoding, wavelet


@dataclasses.dataclass
class Operator:
    """Inputs of one expanded-encoding operator (FP64 arrays)."""
    smaps: np.ndarray      # [C][R]
    coef: np.ndarray       # [T][L]
    time: np.ndarray       # [T]
    basis: np.ndarray      # [L][R]
    dw0: np.ndarray | None # [R]
    n: int                 # image side (R = n*n)

    def A(self, x):
        return encoding.forward(x, self.smaps, self.coef, self.time, self.basis, self.dw0)

    def AH(self, y):
        return encoding.adjoint(y, self.smaps, self.coef, self.time, self.basis, self.dw0)


def pad(x: np.ndarray, n: int, n_pad: int) -> np.ndarray:
    out = np.zeros(x.shape[:-1] + (n_pad, n_pad), dtype=np.complex128)
    out[..., :n, :n] = x.reshape(x.shape[:-1] + (n, n))
    return out


def crop(x: np.ndarray, n: int) -> np.ndarray:
    return x[..., :n, :n].reshape(x.shape[:-2] + (n * n,))


def nrmse(a, ref) -> float:
    return float(np.linalg.norm(np.ravel(a) - np.ravel(ref)) / np.linalg.norm(np.ravel(ref)))


def lambda_rule(op: Operator, y: np.ndarray, factor: float = 1e-3) -> float:
    return float(factor * np.max(np.abs(op.AH(y))))


def objective(op: Operator, y, x_pad, lam: float, levels: int, wname: str) -> float:
    n = op.n
    r = op.A(crop(x_pad, n)) - y
    w = wavelet.dwt2(x_pad, levels, wname)
    det = wavelet.detail_mask(*x_pad.shape[-2:], levels)
    return float(np.vdot(r, r).real + lam * np.sum(np.abs(w[..., det])))


def power_lipschitz(op: Operator, v0: np.ndarray, n_iter: int) -> float:
    """L = 2 * <v, A^H A v> after n_iter normalised power steps from v0."""
    v = v0 / np.linalg.norm(v0)
    for _ in range(n_iter):
        u = op.AH(op.A(v))
        v = u / np.linalg.norm(u)
    return float(2.0 * np.vdot(v, op.AH(op.A(v))).real)


def fista(op: Operator, y, L: float, lam: float, n_iter: int, levels: int, wname: str,
          n_pad: int, ista: bool = False, x0=None, trace: bool = False):
    """Returns crop(x_K) (and the objective after each iteration if trace)."""
    n = op.n
    x_prev = np.zeros((n_pad, n_pad), dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    z = x_prev.copy()
    t = 1.0
    tau = lam / L
    objs = []
    x = x_prev
    for _ in range(n_iter):
        g = 2.0 * pad(op.AH(op.A(crop(z, n)) - y), n, n_pad)
        v = z - g / L
        x = wavelet.idwt2(wavelet.soft_threshold(wavelet.dwt2(v, levels, wname), tau, levels),
                          levels, wname)
        t_next = 1.0 if ista else (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev = x
        t = t_next
        if trace:
            objs.append(objective(op, y, x, lam, levels, wname))
    out = crop(x, n)
    return (out, np.array(objs)) if trace else out


def momentum_coeffs(n_iter: int, ista: bool = False) -> np.ndarray:
    """beta_k = (t_k - 1)/t_{k+1} for k = 1..n_iter."""
    out = []
    t = 1.0
    for _ in range(n_iter):
        tn = 1.0 if ista else (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out.append((t - 1.0) / tn)
        t = tn
    return np.array(out)


def cg_ls(op: Operator, y, n_iter: int) -> np.ndarray:
    """Conjugate gradient on A^H A x = A^H y from x = 0, n_iter iterations."""
    b = op.AH(y)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rs = np.vdot(r, r).real
    for _ in range(n_iter):
        q = op.AH(op.A(p))
        alpha = rs / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rs_new = np.vdot(r, r).real
        p = r + (rs_new / rs) * p
        rs = rs_new
    return x
