"""Pins of the oracle's expanded encoding operator to mathematics that does
not depend on the oracle itself: harmonic-polynomial properties of the
basis, the exact DFT it reduces to on a Cartesian grid, a pure-Python
brute-force summation, the adjoint identity, phase-shift laws and finite
differences of the field-parameter VJPs."""
import cmath

import numpy as np
import pytest

import synth
from oracle import encoding

DEG = synth.SH_DEGREE


def _rand_pts(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.1, 0.1, size=(3, n))


def test_basis_is_harmonic_and_homogeneous():
    x, y, z = _rand_pts(50, 0)
    h = 1e-3
    b0 = encoding.sh_terms(x, y, z)
    lap = (encoding.sh_terms(x + h, y, z) + encoding.sh_terms(x - h, y, z)
           + encoding.sh_terms(x, y + h, z) + encoding.sh_terms(x, y - h, z)
           + encoding.sh_terms(x, y, z + h) + encoding.sh_terms(x, y, z - h) - 6 * b0) / h ** 2
    # cubic polynomials: the central-difference Laplacian is exact up to rounding
    scale = np.max(np.abs(b0), axis=1) / 0.1 ** 2 + 1
    assert np.all(np.max(np.abs(lap), axis=1) / scale < 1e-6)
    for s in (0.5, 2.0, -1.5):
        bs = encoding.sh_terms(s * x, s * y, s * z)
        for l, d in enumerate(DEG):
            np.testing.assert_allclose(bs[l], s ** d * b0[l], rtol=1e-12, atol=1e-15)


def test_basis_spans_harmonics_up_to_third_order():
    # 2d+1 independent homogeneous harmonics per degree: 1, 3, 5, 7
    x, y, z = _rand_pts(200, 1)
    b = encoding.sh_terms(x, y, z)
    for d, cnt in ((0, 1), (1, 3), (2, 5), (3, 7)):
        idx = [l for l, dd in enumerate(DEG) if dd == d]
        assert len(idx) == cnt
        assert np.linalg.matrix_rank(b[idx]) == cnt
    assert encoding.sh_basis(8, 0.2, 0.0, 9).shape == (9, 64)
    assert encoding.sh_basis(8, 0.2, 0.0, 16).shape == (16, 64)


def test_basis_grid_geometry():
    n, fov = 6, 0.3
    b = encoding.sh_basis(n, fov, 0.01, 4)
    dx = fov / n
    # r = j*n + i ; x_i = (i - n/2) dx
    for r in (0, 7, 35):
        j, i = divmod(r, n)
        assert b[1, r] == pytest.approx((i - n / 2) * dx)
        assert b[2, r] == pytest.approx((j - n / 2) * dx)
        assert b[3, r] == pytest.approx(0.01)


@pytest.mark.parametrize("n", [8, 16])
def test_reduces_to_dft_on_cartesian_grid(n):
    fov = 0.2
    coef = synth.cartesian_coef(n, fov, 3)
    basis = encoding.sh_basis(n, fov, 0.0, 3)
    x = synth.random_complex(n * n, 11)
    s = np.ones((1, n * n), dtype=complex)
    y = encoding.forward(x, s, coef, np.zeros(n * n), basis, None)[:, 0].reshape(n, n)
    ref = n * n * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(x.reshape(n, n))))
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < 1e-13
    # adjoint of the unit-coil Cartesian case is the forward DFT
    yy = synth.random_complex((n * n, 1), 12)
    xa = encoding.adjoint(yy, s, coef, np.zeros(n * n), basis, None).reshape(n, n)
    ref_a = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(yy[:, 0].reshape(n, n))))
    assert np.max(np.abs(xa - ref_a)) / np.max(np.abs(ref_a)) < 1e-13


def _small_problem(n=8, c=3, t=64, nbasis=16, seed=5):
    w = synth.Workload("t", n, 0.2, c, t, 4e-6, 2.0, nbasis, 80.0, 20.0, 5, "haar", 1, seed)
    p = synth.make_problem(w)
    basis = encoding.sh_basis(n, w.fov, 0.004, nbasis)
    return p, basis


def _brute_forward(x, smaps, coef, time, basis, dw0):
    t_n, l_n = coef.shape
    c_n, r_n = smaps.shape
    y = np.zeros((t_n, c_n), dtype=complex)
    for t in range(t_n):
        for r in range(r_n):
            ph = dw0[r] * time[t]
            for l in range(l_n):
                ph += coef[t, l] * basis[l, r]
            e = cmath.exp(1j * ph)
            for c in range(c_n):
                y[t, c] += e * smaps[c, r] * x[r]
    return y


def _brute_adjoint(y, smaps, coef, time, basis, dw0):
    t_n, l_n = coef.shape
    c_n, r_n = smaps.shape
    x = np.zeros(r_n, dtype=complex)
    for r in range(r_n):
        for t in range(t_n):
            ph = dw0[r] * time[t]
            for l in range(l_n):
                ph += coef[t, l] * basis[l, r]
            e = cmath.exp(-1j * ph)
            for c in range(c_n):
                x[r] += smaps[c, r].conjugate() * e * y[t, c]
    return x


def test_brute_force_8x8():
    p, basis = _small_problem()
    y = encoding.forward(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0)
    yb = _brute_forward(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0)
    assert np.max(np.abs(y - yb)) / np.max(np.abs(yb)) < 1e-12
    g = synth.random_complex(y.shape, 3)
    x = encoding.adjoint(g, p.smaps, p.coef, p.time, basis, p.dw0)
    xb = _brute_adjoint(g, p.smaps, p.coef, p.time, basis, p.dw0)
    assert np.max(np.abs(x - xb)) / np.max(np.abs(xb)) < 1e-12


def test_single_output_helpers_match_brute_force():
    p, basis = _small_problem(seed=6)
    yb = _brute_forward(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0)
    for t in (0, 17, 63):
        np.testing.assert_allclose(encoding.forward_one(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0, t),
                                   yb[t], rtol=1e-12, atol=1e-12)
    g = synth.random_complex(yb.shape, 4)
    xb = _brute_adjoint(g, p.smaps, p.coef, p.time, basis, p.dw0)
    for r in (0, 9, 63):
        assert abs(encoding.adjoint_one(g, p.smaps, p.coef, p.time, basis, p.dw0, r) - xb[r]) < 1e-11 * np.max(np.abs(xb))


def test_adjoint_identity_and_batch():
    w = synth.TINY
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, 0.0, w.nbasis)
    xs = synth.random_complex((2, w.npix), 21)
    ys = synth.random_complex((2, w.nsamples, w.ncoils), 22)
    ax = encoding.forward(xs, p.smaps, p.coef, p.time, basis, p.dw0)
    ahy = encoding.adjoint(ys, p.smaps, p.coef, p.time, basis, p.dw0)
    for b in range(2):
        lhs = np.vdot(ys[b], ax[b])
        rhs = np.vdot(ahy[b], xs[b])
        assert abs(lhs - rhs) / (np.linalg.norm(ax[b]) * np.linalg.norm(ys[b])) < 1e-13
        # batched call equals single calls
        np.testing.assert_allclose(ax[b], encoding.forward(xs[b], p.smaps, p.coef, p.time, basis, p.dw0),
                                   rtol=0, atol=1e-12 * np.abs(ax).max())


def test_phase_laws():
    p, basis = _small_problem(seed=7)
    args = (p.smaps, p.coef, p.time, basis, p.dw0)
    y0 = encoding.forward(p.x_noisy, *args)
    # constant 0th-order term k0 multiplies every sample by e^{i k0}
    coef = p.coef.copy()
    coef[:, 0] += 0.7
    y1 = encoding.forward(p.x_noisy, p.smaps, coef, p.time, basis, p.dw0)
    np.testing.assert_allclose(y1, np.exp(0.7j) * y0, rtol=1e-12, atol=1e-12)
    # a constant extra off-resonance multiplies y(t) by e^{i dw t}
    y2 = encoding.forward(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0 + 500.0)
    np.testing.assert_allclose(y2, np.exp(1j * 500.0 * p.time)[:, None] * y0, rtol=1e-12, atol=1e-12)
    # shifting a point object by one pixel in x shifts its phase by k_x * dx
    n = 8
    dx = 0.2 / n
    xa = np.zeros(n * n, complex)
    xb = np.zeros(n * n, complex)
    xa[3 * n + 2] = 1.0
    xb[3 * n + 3] = 1.0
    s = p.smaps.copy()
    s[:, 3 * n + 3] = s[:, 3 * n + 2]          # same coil weight at both pixels
    dw = p.dw0.copy()
    dw[3 * n + 3] = dw[3 * n + 2]
    cf = p.coef[:, :3].copy()
    bs = basis[:3]
    ya = encoding.forward(xa, s, cf, p.time, bs, dw)
    yb = encoding.forward(xb, s, cf, p.time, bs, dw)
    np.testing.assert_allclose(yb, np.exp(1j * cf[:, 1] * dx)[:, None] * ya, rtol=1e-12, atol=1e-12)


def test_vjps_match_central_differences():
    p, basis = _small_problem(n=6, c=2, t=20, nbasis=9, seed=8)
    sm, cf, tm, dw = p.smaps, p.coef, p.time, p.dw0
    x = synth.random_complex(36, 31)
    g = synth.random_complex((20, 2), 32)
    gx = synth.random_complex(36, 33)
    yin = synth.random_complex((20, 2), 34)

    def loss_f(xx, cc, dd):
        return float(np.sum((g.conj() * encoding.forward(xx, sm, cc, tm, basis, dd)).real))

    def loss_a(yy, cc, dd):
        return float(np.sum((gx.conj() * encoding.adjoint(yy, sm, cc, tm, basis, dd)).real))

    gxf, gcf, gdf = encoding.vjp_forward(x, g, sm, cf, tm, basis, dw)
    gya, gca, gda = encoding.vjp_adjoint(yin, gx, sm, cf, tm, basis, dw)
    rng = np.random.default_rng(0)
    for _ in range(3):
        dc = rng.normal(size=cf.shape) * 1e-5
        dd = rng.normal(size=dw.shape) * 1e-3
        dxv = (rng.normal(size=36) + 1j * rng.normal(size=36)) * 1e-5
        dyv = (rng.normal(size=(20, 2)) + 1j * rng.normal(size=(20, 2))) * 1e-5
        fd = (loss_f(x + dxv, cf + dc, dw + dd) - loss_f(x - dxv, cf - dc, dw - dd)) / 2
        an = np.sum(gcf * dc) + np.sum(gdf * dd) + np.sum((gxf.conj() * dxv).real)
        assert abs(fd - an) <= 1e-7 * (abs(fd) + 1e-12)
        fd = (loss_a(yin + dyv, cf + dc, dw + dd) - loss_a(yin - dyv, cf - dc, dw - dd)) / 2
        an = np.sum(gca * dc) + np.sum(gda * dd) + np.sum((gya.conj() * dyv).real)
        assert abs(fd - an) <= 1e-7 * (abs(fd) + 1e-12)
