"""Expanded encoding operator (oracle, FP64).  Test infrastructure only.

The paper writes the reconstruction as eq. 1, argmin_x ||A_exp x - y||^2 +
lambda ||W x||_1, and describes A_exp in words (Introduction; Methods 2.1,
2.2.1): a signal model that includes a static B0 map and the dynamic field
measured by probes and fitted to spherical harmonics up to 2nd or 3rd
order, together with the receive-coil sensitivities, for any trajectory.
Written out, for coil c, sample t and pixel r:

    A[(t,c), r] = S_c(r) * exp(i * phi(t, r)),
    phi(t, r)   = sum_l k_l(t) * b_l(r) + dw0(r) * t,

with b_l the real solid harmonics (0th order, x, y, z, five 2nd-order and
seven 3rd-order terms), k_l(t) the monitored coefficient series (terms 1
and 2 are the nominal trajectory k(t)), and dw0 the off-resonance in rad/s.
The exponent sign is +i.  Images are row-major [y][x]; k-space is [T][C].

Everything here is a direct summation of that definition in FP64.  A
library matmul serves for the sum over pixels (forward) or samples
(adjoint); outputs are computed in independent blocks of the output index
only, so no sum is split or reordered.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def sh_terms(x, y, z, nbasis: int = 16) -> np.ndarray:
    """Real solid harmonics at points (x, y, z) (metres), shape [L][P].
    Basis order (unnormalised harmonic polynomials):
      0: 1
      1: x   2: y   3: z
      4: xy  5: yz  6: 2z^2-x^2-y^2  7: xz  8: x^2-y^2
      9: 3x^2y-y^3  10: xyz  11: y(4z^2-x^2-y^2)  12: z(2z^2-3x^2-3y^2)
      13: x(4z^2-x^2-y^2)  14: z(x^2-y^2)  15: x^3-3xy^2
    Orders up to 2 use the first 9 terms, up to 3 all 16 (Introduction:
    fields expanded in spherical harmonics up to 2nd or 3rd order)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64) + np.zeros_like(x)
    terms = [
        np.ones_like(x),
        x, y, z,
        x * y, y * z, 2 * z * z - x * x - y * y, x * z, x * x - y * y,
        3 * x * x * y - y ** 3, x * y * z, y * (4 * z * z - x * x - y * y),
        z * (2 * z * z - 3 * x * x - 3 * y * y), x * (4 * z * z - x * x - y * y),
        z * (x * x - y * y), x ** 3 - 3 * x * y * y,
    ]
    if not 0 <= nbasis <= 16:
        raise ValueError("nbasis must be in [0, 16]")
    return np.stack(terms[:nbasis]) if nbasis else np.zeros((0,) + x.shape)


def sh_basis(n: int, fov: float, z0: float = 0.0, nbasis: int = 16, ny: int | None = None,
             fov_y: float | None = None) -> np.ndarray:
    """b_l(r) on the pixel grid, shape [L][R]: pixel centres
    x_i = (i - nx/2) * fov/nx (likewise y), slice at z = z0, r = j*nx + i."""
    nx = n
    ny = n if ny is None else ny
    fx = fov
    fy = fov if fov_y is None else fov_y
    xs = (np.arange(nx) - nx / 2) * (fx / nx)
    ys = (np.arange(ny) - ny / 2) * (fy / ny)
    y, x = np.meshgrid(ys, xs, indexing="ij")
    return sh_terms(x.reshape(-1), y.reshape(-1), z0, nbasis)


def phase(coef: np.ndarray, time: np.ndarray, basis: np.ndarray, dw0) -> np.ndarray:
    """phi(t, r) = sum_l k_l(t) b_l(r) + dw0(r) t, shape [T][R] (rad)."""
    ph = coef @ basis if basis.shape[0] else np.zeros((coef.shape[0], basis.shape[1]))
    if dw0 is not None:
        ph = ph + np.outer(time, dw0)
    return ph


def _blocks(n: int, size: int):
    return [(s, min(s + size, n)) for s in range(0, n, size)]


def _pool():
    return ThreadPoolExecutor(max_workers=int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1)))


def forward(x, smaps, coef, time, basis, dw0=None, block: int = 512) -> np.ndarray:
    """y = A_exp x.  x: [R] or [B][R]; returns [T][C] or [B][T][C].

    y[b, t, c] = sum_r exp(i phi(t, r)) * S_c(r) * x_b(r)."""
    x = np.asarray(x, dtype=np.complex128)
    single = x.ndim == 1
    xb = x[None] if single else x
    nb, r_n = xb.shape
    c_n = smaps.shape[0]
    t_n = coef.shape[0]
    # Z[r, (b, c)] = S_c(r) x_b(r)
    z = (xb[:, None, :] * smaps[None, :, :]).reshape(nb * c_n, r_n).T
    y = np.empty((t_n, nb * c_n), dtype=np.complex128)

    def run(se):
        s, e = se
        e_blk = np.exp(1j * phase(coef[s:e], time[s:e], basis, dw0))
        y[s:e] = e_blk @ z

    with _pool() as p:
        list(p.map(run, _blocks(t_n, block)))
    y = y.reshape(t_n, nb, c_n).transpose(1, 0, 2)
    return y[0] if single else y


def adjoint(y, smaps, coef, time, basis, dw0=None, block: int = 256) -> np.ndarray:
    """x = A_exp^H y.  y: [T][C] or [B][T][C]; returns [R] or [B][R].

    x[b, r] = sum_c conj(S_c(r)) sum_t conj(exp(i phi(t, r))) y[b, t, c]."""
    y = np.asarray(y, dtype=np.complex128)
    single = y.ndim == 2
    yb = y[None] if single else y
    nb, t_n, c_n = yb.shape
    r_n = smaps.shape[1]
    ymat = yb.transpose(1, 0, 2).reshape(t_n, nb * c_n)
    xc = np.empty((r_n, nb * c_n), dtype=np.complex128)

    def run(se):
        s, e = se
        d = None if dw0 is None else dw0[s:e]
        e_blk = np.exp(1j * phase(coef, time, basis[:, s:e], d))   # [T][Rblk]
        xc[s:e] = e_blk.conj().T @ ymat

    with _pool() as p:
        list(p.map(run, _blocks(r_n, block)))
    xc = xc.reshape(r_n, nb, c_n)
    x = np.einsum("rbc,cr->br", xc, smaps.conj())
    return x[0] if single else x


def forward_one(x, smaps, coef, time, basis, dw0, t: int) -> np.ndarray:
    """One k-space sample y[t, :] (all coils) by direct summation; used to
    check single outputs of full-size GPU runs."""
    ph = coef[t] @ basis + (0.0 if dw0 is None else time[t] * dw0)
    e = np.exp(1j * ph)
    return (smaps * (e * x)[None, :]).sum(axis=1)


def adjoint_one(y, smaps, coef, time, basis, dw0, r: int) -> complex:
    """One image pixel x[r] of A^H y by direct summation."""
    ph = coef @ basis[:, r] + (0.0 if dw0 is None else time * dw0[r])
    e = np.exp(1j * ph)
    return complex(np.sum(smaps[:, r].conj() * (e.conj() @ y)))


# ---------------------------------------------------------------------------
# Vector-Jacobian products with respect to the field parameters.  Real
# parameters theta get d(loss)/d(theta); complex tensors use the convention
# grad = dL/dRe + i dL/dIm.  Derived from dA/dk_l(t) = i b_l(r) A and
# dA/d dw0(r) = i t A applied to the entry formula above.
# ---------------------------------------------------------------------------

def vjp_forward(x, g, smaps, coef, time, basis, dw0):
    """For y = A x with upstream g = dL/dy ([T][C]): returns
    (grad_x [R], grad_coef [T][L], grad_dw0 [R]).

      grad_x              = A^H g
      grad_coef[t, l]     = -Im sum_c conj(g[t,c]) (E (b_l * Z))[t, c]
      grad_dw0[r]         = -Im sum_c Z[r,c] conj((E^H (t * g))[r, c])
    with Z = S x and E[t, r] = exp(i phi)."""
    ph = phase(coef, time, basis, dw0)
    e = np.exp(1j * ph)
    z = (smaps * x[None, :]).T                          # [R][C]
    grad_x = adjoint(g, smaps, coef, time, basis, dw0)
    gc = np.empty(coef.shape)
    for l in range(basis.shape[0]):
        yl = e @ (basis[l][:, None] * z)                # [T][C]
        gc[:, l] = -np.imag(np.sum(g.conj() * yl, axis=1))
    eh_tg = e.conj().T @ (time[:, None] * g)            # [R][C]
    gd = -np.imag(np.sum(z * eh_tg.conj(), axis=1))
    return grad_x, gc, gd


def vjp_adjoint(y, gx, smaps, coef, time, basis, dw0):
    """For x = A^H y with upstream gx = dL/dx ([R]): returns
    (grad_y [T][C], grad_coef [T][L], grad_dw0 [R]).

      grad_y          = A gx
      grad_coef[t, l] = Im sum_c y[t,c] conj((E (b_l * S * gx))[t, c])
      grad_dw0[r]     = Im( conj(gx[r]) sum_c conj(S_c(r)) (E^H (t * y))[r, c] )"""
    ph = phase(coef, time, basis, dw0)
    e = np.exp(1j * ph)
    grad_y = forward(gx, smaps, coef, time, basis, dw0)
    sg = (smaps * gx[None, :]).T                         # [R][C]
    gc = np.empty(coef.shape)
    for l in range(basis.shape[0]):
        yl = e @ (basis[l][:, None] * sg)
        gc[:, l] = np.imag(np.sum(y * yl.conj(), axis=1))
    eh_ty = e.conj().T @ (time[:, None] * y)             # [R][C]
    gd = np.imag(gx.conj() * np.sum(smaps.conj().T * eh_ty, axis=1))
    return grad_y, gc, gd



# The same field-parameter VJPs without forming E whole (for sizes such as
# 128 x 128 pixels x 12000 samples): grad_coef is computed in blocks of its
# sample index t, grad_dw0 in blocks of its pixel index r, each block by the
# formulas above restricted to its own outputs (no sum is split).

def _basis_products(e_blk, basis, z):
    """(E_blk (b_l * z))[t, l, c] for every basis term l: one matmul with the
    L*C columns b_l(r) z[r, c]."""
    r_n, c_n = z.shape
    l_n = basis.shape[0]
    bz = (basis[:, :, None] * z[None, :, :]).transpose(1, 0, 2).reshape(r_n, l_n * c_n)
    return (e_blk @ bz).reshape(e_blk.shape[0], l_n, c_n)


def field_vjp_forward(x, g, smaps, coef, time, basis, dw0, block: int = 256):
    """(grad_coef [T][L], grad_dw0 [R] or None) of vjp_forward, blocked:
      grad_coef[t, l] = -Im sum_c conj(g[t,c]) (E (b_l * Z))[t, c]   (blocks of t)
      grad_dw0[r]     = -Im sum_c Z[r,c] conj((E^H (t * g))[r, c])   (blocks of r)"""
    g = np.asarray(g, dtype=np.complex128)
    z = (smaps * np.asarray(x, dtype=np.complex128)[None, :]).T      # [R][C]
    t_n, r_n = coef.shape[0], smaps.shape[1]
    gc = np.empty(coef.shape)
    gd = None if dw0 is None else np.empty(r_n)

    def run_t(se):
        s, e = se
        e_blk = np.exp(1j * phase(coef[s:e], time[s:e], basis, dw0))            # [Tblk][R]
        gc[s:e] = -np.imag(np.sum(g[s:e, None, :].conj() * _basis_products(e_blk, basis, z), axis=2))

    def run_r(se):
        s, e = se
        e_blk = np.exp(1j * phase(coef, time, basis[:, s:e], dw0[s:e]))          # [T][Rblk]
        eh_tg = e_blk.conj().T @ (time[:, None] * g)                             # [Rblk][C]
        gd[s:e] = -np.imag(np.sum(z[s:e] * eh_tg.conj(), axis=1))

    with _pool() as p:
        list(p.map(run_t, _blocks(t_n, block)))
        if dw0 is not None:
            list(p.map(run_r, _blocks(r_n, block)))
    return gc, gd


def field_vjp_adjoint(y, gx, smaps, coef, time, basis, dw0, block: int = 256):
    """(grad_coef [T][L], grad_dw0 [R] or None) of vjp_adjoint, blocked:
      grad_coef[t, l] = Im sum_c y[t,c] conj((E (b_l * S * gx))[t, c])             (blocks of t)
      grad_dw0[r]     = Im( conj(gx[r]) sum_c conj(S_c(r)) (E^H (t * y))[r, c] )   (blocks of r)"""
    y = np.asarray(y, dtype=np.complex128)
    gx = np.asarray(gx, dtype=np.complex128)
    sg = (smaps * gx[None, :]).T                                              # [R][C]
    t_n, r_n = coef.shape[0], smaps.shape[1]
    gc = np.empty(coef.shape)
    gd = None if dw0 is None else np.empty(r_n)

    def run_t(se):
        s, e = se
        e_blk = np.exp(1j * phase(coef[s:e], time[s:e], basis, dw0))
        gc[s:e] = np.imag(np.sum(y[s:e, None, :] * _basis_products(e_blk, basis, sg).conj(), axis=2))

    def run_r(se):
        s, e = se
        e_blk = np.exp(1j * phase(coef, time, basis[:, s:e], dw0[s:e]))
        eh_ty = e_blk.conj().T @ (time[:, None] * y)
        gd[s:e] = np.imag(gx[s:e].conj() * np.sum(smaps[:, s:e].conj().T * eh_ty, axis=1))

    with _pool() as p:
        list(p.map(run_t, _blocks(t_n, block)))
        if dw0 is not None:
            list(p.map(run_r, _blocks(r_n, block)))
    return gc, gd
