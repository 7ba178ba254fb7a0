"""Pins of the oracle's solvers: the closed-form FISTA solution on an
orthogonal (fully sampled Cartesian) encoding, the exact Lipschitz
constant, ISTA monotone descent, the FISTA O(1/k^2) rate bound, the KKT
conditions at a long-run optimum, CG against a dense least-squares solve,
and the bf16/fp16 rounding emulation against torch's conversions."""
import math

import numpy as np
import pytest

import synth
from oracle import encoding, solve, splitemu, wavelet


def _cartesian_op(n=16, c=4, normalise=True, seed=0):
    fov = 0.2
    w = synth.Workload("cart", n, fov, c, n * n, 1e-6, 1.0, 3, 0.0, 20.0, 5, "haar", 2, seed)
    s = synth.coil_maps(w)
    if normalise:
        s = s / np.sqrt(np.sum(np.abs(s) ** 2, axis=0))[None, :]
    coef = synth.cartesian_coef(n, fov, 3)
    basis = encoding.sh_basis(n, fov, 0.0, 3)
    return solve.Operator(s, coef, np.zeros(n * n), basis, None, n), w


def test_cartesian_gram_and_power_iteration():
    op, w = _cartesian_op(normalise=False)
    n = op.n
    # A^H A = N^2 diag(sum_c |S_c|^2): max eigenvalue N^2 * max_r sum|S|^2 (= N^2 here)
    v0 = synth.power_start(n * n, 1)
    L = solve.power_lipschitz(op, v0, 400)
    lam_max = n * n * np.max(np.sum(np.abs(op.smaps) ** 2, axis=0))
    assert L == pytest.approx(2 * lam_max, rel=2e-3)
    assert L <= 2 * lam_max * (1 + 1e-12)


def _dense(op):
    r = op.n * op.n
    cols = [op.A(np.eye(r)[i]).reshape(-1) for i in range(r)]
    return np.stack(cols, axis=1)


def test_power_iteration_matches_eigvalsh_8x8():
    n = 8
    w = synth.Workload("p", n, 0.2, 2, 48, 4e-6, 2.0, 9, 60.0, 20.0, 5, "haar", 1, 3)
    p = synth.make_problem(w)
    op = solve.Operator(p.smaps, p.coef, p.time, encoding.sh_basis(n, w.fov, 0.0, 9), p.dw0, n)
    a = _dense(op)
    ev = np.linalg.eigvalsh(a.conj().T @ a)
    L = solve.power_lipschitz(op, synth.power_start(n * n, 2), 300)
    assert L == pytest.approx(2 * ev[-1], rel=1e-6)


def test_fista_closed_form_on_orthogonal_encoding():
    op, w = _cartesian_op()
    n = op.n
    x = synth.phantom(synth.Workload("c", n, 0.2, 4, n * n, 1e-6, 1, 3, 0, 20, 5, "haar", 2, 4))
    y = op.A(x) + 0.01 * synth.random_complex((n * n, op.smaps.shape[0]), 5)
    L = 2.0 * n * n                          # A^H A = N^2 I exactly
    lam = solve.lambda_rule(op, y, 0.05)
    levels = 2
    # x_hat = W^H S_{lam/(2N^2)}(W A^H y / N^2): the fixed point reached at k = 1
    ahy = solve.pad(op.AH(y), n, n)
    expect = wavelet.idwt2(wavelet.soft_threshold(wavelet.dwt2(ahy / (n * n), levels, "haar"),
                                                  lam / L, levels), levels, "haar")
    for k in (1, 2, 7):
        got = solve.fista(op, y, L, lam, k, levels, "haar", n)
        assert np.max(np.abs(got - expect.reshape(-1))) < 1e-12 * np.max(np.abs(expect))


def _small_cs(seed=9, n=8):
    w = synth.Workload("s", n, 0.2, 3, 96, 4e-6, 2.0, 9, 60.0, 15.0, 5, "haar", 1, seed)
    p = synth.make_problem(w)
    op = solve.Operator(p.smaps, p.coef, p.time, encoding.sh_basis(n, w.fov, 0.0, 9), p.dw0, n)
    y = op.A(p.x_noisy)
    L = solve.power_lipschitz(op, synth.power_start(n * n, 3), 200) * 1.0001
    lam = solve.lambda_rule(op, y, 0.05)
    return op, y, L, lam


def test_ista_monotone_and_fista_rate_bound():
    op, y, L, lam = _small_cs()
    n = op.n
    _, f_ista = solve.fista(op, y, L, lam, 30, 1, "haar", n, ista=True, trace=True)
    assert np.all(np.diff(f_ista) <= 1e-12 * f_ista[0])
    x_star, f_long = solve.fista(op, y, L, lam, 3000, 1, "haar", n, trace=True)
    f_star = f_long[-1]
    _, f_k = solve.fista(op, y, L, lam, 40, 1, "haar", n, trace=True)
    r0 = np.linalg.norm(solve.pad(x_star, n, n)) ** 2      # x0 = 0
    for k, fk in enumerate(f_k, start=1):
        assert fk - f_star <= 2 * L * r0 / (k + 1) ** 2 * (1 + 1e-9) + 1e-12
    f0 = solve.objective(op, y, np.zeros((n, n), complex), lam, 1, "haar")
    assert f_k[-1] < f0


def test_kkt_at_long_run_optimum():
    op, y, L, lam = _small_cs(seed=10)
    n = op.n
    x = solve.fista(op, y, L, lam, 6000, 1, "haar", n)
    xp = solve.pad(x, n, n)
    grad = 2 * solve.pad(op.AH(op.A(x) - y), n, n)
    q = wavelet.dwt2(grad, 1, "haar")
    wx = wavelet.dwt2(xp, 1, "haar")
    det = wavelet.detail_mask(n, n, 1)
    tol = 1e-6 * lam
    assert np.max(np.abs(q[~det])) < tol * 10
    for qi, wi in zip(q[det], wx[det]):
        if abs(wi) > 1e-9:
            assert abs(qi + lam * wi / abs(wi)) < tol * 10
        else:
            assert abs(qi) <= lam * (1 + 1e-6)


def test_cg_matches_least_squares():
    n = 6
    w = synth.Workload("cg", n, 0.2, 2, 60, 4e-6, 2.0, 9, 60.0, 20.0, 5, "haar", 1, 12)
    p = synth.make_problem(w)
    op = solve.Operator(p.smaps, p.coef, p.time, encoding.sh_basis(n, w.fov, 0.0, 9), p.dw0, n)
    y = op.A(p.x_noisy) + 0.05 * synth.random_complex((60, 2), 13)
    a = _dense(op)
    ref = np.linalg.lstsq(a, y.reshape(-1), rcond=None)[0]
    x = solve.cg_ls(op, y, 200)
    assert solve.nrmse(x, ref) < 1e-6
    # orthogonal case: one CG step is exact
    op2, _ = _cartesian_op(n=8)
    y2 = synth.random_complex((64, 4), 14)
    np.testing.assert_allclose(solve.cg_ls(op2, y2, 1), op2.AH(y2) / 64, atol=1e-12)


def test_nrmse_and_lambda_rule():
    a = np.array([1.0, 2.0, 2.0])
    assert solve.nrmse(a * 1.1, a) == pytest.approx(0.1)
    op, w = _cartesian_op(n=8)
    y = synth.random_complex((64, 4), 15)
    assert solve.lambda_rule(op, y) == pytest.approx(1e-3 * np.max(np.abs(op.AH(y))))


def test_momentum_coefficients():
    b = solve.momentum_coeffs(5)
    assert b[0] == 0.0
    t = [1.0]
    for _ in range(5):
        t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    np.testing.assert_allclose(b, [(t[k] - 1) / t[k + 1] for k in range(5)])
    assert np.all(solve.momentum_coeffs(4, ista=True) == 0)


def test_split_rounding_matches_torch_and_error_level():
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(1).normal(size=4096).astype(np.float32) * 3
    ref_bf = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(splitemu.round_bf16(v), ref_bf)
    ref_h = torch.from_numpy(v).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(splitemu.round_fp16(v), ref_h)
    rng = np.random.default_rng(2)
    ph = rng.uniform(-300, 300, size=(128, 1024))
    e = np.exp(1j * ph)
    z = rng.normal(size=(1024, 8)) + 1j * rng.normal(size=(1024, 8))
    ref = e @ z
    err_bf = np.linalg.norm(splitemu.split_cmatmul(e, z, "bf16") - ref) / np.linalg.norm(ref)
    err_h = np.linalg.norm(splitemu.split_cmatmul(e, z, "fp16") - ref) / np.linalg.norm(ref)
    assert 1e-7 < err_bf < 2e-5      # about 3 * 2^-16 per product, averaged
    assert err_h < 1e-6
