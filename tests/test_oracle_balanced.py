"""Pins of the undecimated-wavelet / sigma-weight / balanced-FISTA oracle
(CPU): tight-frame identity, energy, adjointness and the Haar closed form of
the transform (odd and even sizes); constant images; the histogram mode of
Rayleigh samples; the closed-form minimiser of the balanced model when
A^H A = c I and kappa = 2c (which makes the smooth part c ||alpha - W x0||^2);
monotone ISTA objective on a general encoding."""
import numpy as np
import pytest

import synth
from oracle import balanced as bal
from oracle import encoding, solve


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("name", ["haar", "db4"])
@pytest.mark.parametrize("n,levels", [(12, 1), (13, 2), (16, 3)])
def test_tight_frame_energy_and_adjoint(name, n, levels):
    rng = np.random.default_rng(n + levels)
    x = _crandn(rng, n, n)
    w = bal.swt2(x, levels, name)
    assert w.shape == (3 * levels + 1, n, n)
    assert np.linalg.norm(bal.iswt2(w, levels, name) - x) <= 1e-12 * np.linalg.norm(x)
    assert abs(np.linalg.norm(w) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    v = _crandn(rng, *w.shape)
    lhs = np.vdot(v, w)
    rhs = np.vdot(bal.iswt2(v, levels, name), x)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(v) * np.linalg.norm(x)


def test_haar_level_one_closed_form():
    rng = np.random.default_rng(3)
    u = _crandn(rng, 7, 9)[:7, :7]
    w = bal.swt2(u, 1, "haar")
    i, j = 2, 5
    a, b = u[i, j], u[i, (j + 1) % 7]
    c, d = u[(i + 1) % 7, j], u[(i + 1) % 7, (j + 1) % 7]
    assert np.isclose(w[0, i, j], ((a - b) + (c - d)) / 4)      # high x, low y
    assert np.isclose(w[1, i, j], ((a + b) - (c + d)) / 4)      # low x, high y
    assert np.isclose(w[2, i, j], ((a - b) - (c - d)) / 4)      # high x, high y
    assert np.isclose(w[3, i, j], (a + b + c + d) / 4)          # low pass


@pytest.mark.parametrize("name", ["haar", "db4"])
def test_constant_image_has_no_details(name):
    w = bal.swt2(np.full((10, 10), 2.0 - 1.0j), 2, name)
    assert np.max(np.abs(w[:6])) <= 1e-13
    assert np.allclose(w[6], 2.0 - 1.0j, atol=1e-13)


def test_histogram_mode_of_rayleigh_samples():
    rng = np.random.default_rng(4)
    sigma = 2.5
    z = sigma * (rng.standard_normal(1_000_000) + 1j * rng.standard_normal(1_000_000))
    est = bal.histogram_mode(np.abs(z))
    assert abs(est - sigma) <= 0.15 * sigma
    # the weights: sigma/2 per level on the high-pass bands, 0 on the low pass
    w = np.stack([z[:10000].reshape(100, 100)] * 4)
    lam = bal.sigma_weights(w, 1)
    assert lam[3] == 0.0 and lam[0] == lam[1] == lam[2] > 0


@pytest.mark.parametrize("name,levels", [("haar", 1), ("db4", 1), ("db4", 2)])
def test_balanced_closed_form_for_unitary_encoding(name, levels):
    n = 8
    coef = synth.cartesian_coef(n, 0.2)
    tm = np.zeros(coef.shape[0])
    basis = encoding.sh_basis(n, 0.2, 0.0, coef.shape[1])
    op = solve.Operator(np.ones((1, n * n), complex), coef, tm, basis, None, n)
    rng = np.random.default_rng(5)
    x0 = _crandn(rng, n * n)
    y = op.A(x0)
    c = float(np.real(np.vdot(x0, op.AH(op.A(x0))) / np.vdot(x0, x0)))   # A^H A = c I
    assert np.allclose(op.AH(op.A(x0)), c * x0, rtol=1e-10)
    lam = np.full(3 * levels + 1, 0.3 * c)
    lam[-1] = 0.0
    x = bal.fista(op, y, 2 * c, 2 * c, lam, 150, levels, name)
    ref = bal.iswt2(bal.soft_bands(bal.swt2(x0.reshape(n, n), levels, name), lam / (2 * c)), levels, name)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_balanced_ista_objective_decreases():
    w = synth.Workload("bal", 12, 0.2, 3, 300, 3e-6, 2.0, 9, 60.0, 20.0, 8, "db4", 1, 31)
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, 0.0, w.nbasis)
    op = solve.Operator(p.smaps, p.coef, p.time, basis, p.dw0, w.n)
    y = op.A(p.x_noisy)
    L_A = 1.01 * solve.power_lipschitz(op, synth.power_start(w.npix, 1), 50)
    lam = bal.sigma_weights(bal.swt2(op.AH(y).reshape(w.n, w.n), 1, "db4"), 1)
    _, f = bal.fista(op, y, L_A, L_A, lam, 15, 1, "db4", ista=True, trace=True)
    assert np.all(np.diff(f) <= 1e-9 * f[0])
