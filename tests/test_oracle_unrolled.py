"""Pins of the oracle's unrolled-FISTA gradients (torch float64 autograd)
against central finite differences of the independent NumPy FISTA loss."""
import numpy as np
import pytest

import synth
from oracle import encoding, solve, unrolled


def _setup(seed=5):
    w = synth.Workload("u", 8, 0.2, 2, 80, 4e-6, 2.0, 9, 60.0, 15.0, 4, "haar", 1, seed)
    p = synth.make_problem(w)
    basis = encoding.sh_basis(8, 0.2, 0.002, 9)
    op = solve.Operator(p.smaps, p.coef, p.time, basis, p.dw0, 8)
    L = 1.01 * solve.power_lipschitz(op, synth.power_start(64, 1), 50)
    lam = solve.lambda_rule(op, op.A(p.x_noisy), 0.05)
    return w, p, basis, L, lam


def _numpy_loss(w, p, basis, L, lam, x_in, coef, dw0):
    op = solve.Operator(p.smaps, coef, p.time, basis, dw0, w.n)
    xh = solve.fista(op, op.A(x_in), L, lam, 4, 1, "haar", 8)
    return float(np.sum(np.abs(xh - p.x_true) ** 2))


def test_unrolled_gradients_match_central_differences():
    w, p, basis, L, lam = _setup()
    loss, gx, gc, gd = unrolled.loss_and_grads(p.x_noisy, p.x_true, p.smaps, p.coef, p.time, basis, p.dw0, L, lam,
                                               4, 1, "haar", 8, 8)
    assert loss == pytest.approx(_numpy_loss(w, p, basis, L, lam, p.x_noisy, p.coef, p.dw0), rel=1e-12)
    rng = np.random.default_rng(3)
    errs = []
    for _ in range(5):
        h = 1e-6
        dx = (rng.normal(size=64) + 1j * rng.normal(size=64)) * h
        dc = rng.normal(size=p.coef.shape) * h * np.max(np.abs(p.coef))
        dd = rng.normal(size=64) * h * 100.0
        fp = _numpy_loss(w, p, basis, L, lam, p.x_noisy + dx, p.coef + dc, p.dw0 + dd)
        fm = _numpy_loss(w, p, basis, L, lam, p.x_noisy - dx, p.coef - dc, p.dw0 - dd)
        fd = (fp - fm) / 2
        an = np.sum((gx.conj() * dx).real) + np.sum(gc * dc) + np.sum(gd * dd)
        errs.append(abs(fd - an) / max(abs(fd), 1e-30))
    # soft-threshold kinks can spoil a single direction; the median must agree
    assert np.median(errs) < 1e-5


def test_blocked_field_vjps_equal_the_unblocked_ones():
    w = synth.Workload("v", 9, 0.2, 3, 70, 4e-6, 2.0, 16, 60.0, 15.0, 4, "haar", 1, 5)
    p = synth.make_problem(w)
    b = encoding.sh_basis(9, 0.2, 0.003, 16)
    args = (p.smaps, p.coef, p.time, b, p.dw0)
    g = synth.random_complex((70, 3), 3)
    gx = synth.random_complex(81, 4)
    _, c1, d1 = encoding.vjp_forward(p.x_noisy, g, *args)
    c2, d2 = encoding.field_vjp_forward(p.x_noisy, g, *args, block=16)
    np.testing.assert_allclose(c2, c1, rtol=0, atol=1e-12 * np.max(np.abs(c1)))
    np.testing.assert_allclose(d2, d1, rtol=0, atol=1e-12 * np.max(np.abs(d1)))
    _, c1, d1 = encoding.vjp_adjoint(g, gx, *args)
    c2, d2 = encoding.field_vjp_adjoint(g, gx, *args, block=16)
    np.testing.assert_allclose(c2, c1, rtol=0, atol=1e-12 * np.max(np.abs(c1)))
    np.testing.assert_allclose(d2, d1, rtol=0, atol=1e-12 * np.max(np.abs(d1)))


def test_reverse_pass_matches_autograd_16px():
    """The hand-written reverse pass against torch's autograd of the
    independent torch FISTA (16 x 16, 4 coils, 400 samples, 16 field terms +
    dB0, 5 iterations, db4 J = 2): two derivations of one gradient."""
    w = synth.Workload("unr", 16, 0.2, 4, 400, 4e-6, 2.0, 16, 80.0, 15.0, 5, "db4", 2, 81)
    p = synth.make_problem(w)
    basis = encoding.sh_basis(16, 0.2, 0.003, 16)
    op = solve.Operator(p.smaps, p.coef, p.time, basis, p.dw0, 16)
    L = 1.01 * solve.power_lipschitz(op, synth.power_start(256, 2), 60)
    lam = solve.lambda_rule(op, op.A(p.x_noisy), 0.02)
    args = (p.x_noisy, p.x_true, p.smaps, p.coef, p.time, basis, p.dw0, L, lam, 5, 2, "db4", 16, 16)
    l1, gx1, gc1, gd1 = unrolled.loss_and_grads(*args)
    l2, gx2, gc2, gd2 = unrolled.reverse_loss_and_grads(*args)
    assert l2 == pytest.approx(l1, rel=1e-12)
    for a, b in ((gx2, gx1), (gc2, gc1), (gd2, gd1)):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


def test_reverse_pass_matches_central_differences():
    w, p, basis, L, lam = _setup(seed=6)
    loss, gx, gc, gd = unrolled.reverse_loss_and_grads(p.x_noisy, p.x_true, p.smaps, p.coef, p.time, basis, p.dw0,
                                                       L, lam, 4, 1, "haar", 8, 8)
    assert loss == pytest.approx(_numpy_loss(w, p, basis, L, lam, p.x_noisy, p.coef, p.dw0), rel=1e-12)
    rng = np.random.default_rng(4)
    errs = []
    for _ in range(5):
        h = 1e-6
        dx = (rng.normal(size=64) + 1j * rng.normal(size=64)) * h
        dc = rng.normal(size=p.coef.shape) * h * np.max(np.abs(p.coef))
        dd = rng.normal(size=64) * h * 100.0
        fp = _numpy_loss(w, p, basis, L, lam, p.x_noisy + dx, p.coef + dc, p.dw0 + dd)
        fm = _numpy_loss(w, p, basis, L, lam, p.x_noisy - dx, p.coef - dc, p.dw0 - dd)
        fd = (fp - fm) / 2
        an = np.sum((gx.conj() * dx).real) + np.sum(gc * dc) + np.sum(gd * dd)
        errs.append(abs(fd - an) / max(abs(fd), 1e-30))
    assert np.median(errs) < 1e-5
