"""Pins of the oracle's solvers: the closed-form FISTA solution on an
orthogonal (fully sampled Cartesian) encoding, the exact Lipschitz
constant, ISTA monotone descent, the FISTA O(1/k^2) rate bound, the KKT
conditions at a long-run optimum, CG against a dense least-squares solve,
the objective of eq. 1 against its closed-form minimum (with mutants that
must fail), the lambda rule on a point object, and the bf16/fp16 rounding
emulation against torch's conversions."""
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


def test_nrmse():
    a = np.array([1.0, 2.0, 2.0])
    assert solve.nrmse(a * 1.1, a) == pytest.approx(0.1)


def test_lambda_rule_point_object():
    """Unit coil, full Cartesian sampling: A^H A = N^2 I, so for a point object
    a*delta_r the zero-filled image A^H y is N^2 a delta_r and the rule gives
    lambda = 1e-3 * N^2 |a| (the lambda of Methods 2.1 read from W A^T y)."""
    n = 8
    fov = 0.2
    coef = synth.cartesian_coef(n, fov, 3)
    op = solve.Operator(np.ones((1, n * n), complex), coef, np.zeros(n * n), encoding.sh_basis(n, fov, 0.0, 3),
                        None, n)
    for r, a in ((0, 1.0), (27, 0.3 - 2.0j), (63, -5.5j)):
        x = np.zeros(n * n, complex)
        x[r] = a
        assert solve.lambda_rule(op, op.A(x)) == pytest.approx(1e-3 * n * n * abs(a), rel=1e-12)
        assert solve.lambda_rule(op, op.A(x), 0.05) == pytest.approx(0.05 * n * n * abs(a), rel=1e-12)


def _orthogonal_problem(n=16, levels=2, seed=21):
    """Cartesian encoding with sum_c |S_c|^2 = 1 (A^H A = N^2 I), data, lambda
    and the closed-form minimiser of eq. 1: with u = A^H y / N^2,
    ||A x - y||^2 = N^2 ||x - u||^2 + ||y||^2 - N^2 ||u||^2 and W orthonormal,
    so w_hat = S_{lambda/(2 N^2)}(W u) on the detail bands, (W u) on LL."""
    op, _ = _cartesian_op(n=n, seed=seed)
    x = synth.phantom(synth.Workload("o", n, 0.2, 4, n * n, 1e-6, 1, 3, 0, 20, 5, "haar", levels, seed + 1))
    y = op.A(x) + 0.02 * synth.random_complex((n * n, op.smaps.shape[0]), seed + 2)
    lam = 0.08 * np.max(np.abs(op.AH(y)))
    u = solve.pad(op.AH(y) / (n * n), n, n)
    wu = wavelet.dwt2(u, levels, "haar")
    det = wavelet.detail_mask(n, n, levels)
    w_hat = wu.copy()
    mag = np.abs(wu[det])
    t = lam / (2 * n * n)
    w_hat[det] = np.where(mag > t, wu[det] * (1 - t / np.maximum(mag, 1e-300)), 0)
    x_hat = wavelet.idwt2(w_hat, levels, "haar")
    # the minimum value from the decomposition above (no call of the objective)
    f_min = (np.vdot(y, y).real - n * n * np.vdot(u, u).real + n * n * np.sum(np.abs(w_hat - wu) ** 2)
             + lam * np.sum(np.abs(w_hat[det])))
    return op, y, lam, levels, x_hat, f_min


def _minimiser_holds(objective, op, y, lam, levels, x_hat, f_min):
    """True iff the objective takes the closed-form minimum value at x_hat and
    no pair of perturbations +-delta lowers it: 24 random image-domain
    directions, 24 random directions on the support of W x_hat (where the l1
    term is differentiable) and the ray through x_hat, at three scales."""
    n = op.n
    f_hat = objective(op, y, x_hat, lam, levels, "haar")
    if abs(f_hat - f_min) > 1e-10 * abs(f_min):
        return False
    rng = np.random.default_rng(5)
    supp = np.abs(wavelet.dwt2(x_hat, levels, "haar")) > 0
    dirs = []
    for k in range(24):
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        dirs.append((k, d))
        e = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * supp
        dirs.append((k, wavelet.idwt2(e, levels, "haar")))
    dirs += [(k, x_hat) for k in range(3)]
    for k, d in dirs:
        d = d * 10.0 ** (-2 - k % 3) * np.linalg.norm(x_hat) / np.linalg.norm(d)
        for sgn in (1.0, -1.0):
            if objective(op, y, x_hat + sgn * d, lam, levels, "haar") < f_hat - 1e-13 * abs(f_hat):
                return False
    return True


def test_objective_pins():
    """solve.objective is eq. 1 as written: F(0) = ||y||^2, and on an
    orthogonal encoding it takes the closed-form minimum at the closed-form
    minimiser and rises along every tested direction.  The same check rejects
    plausible mistakes: a 1/2 on the data term, a penalised LL band, squared
    moduli in the l1 term."""
    op, y, lam, levels, x_hat, f_min = _orthogonal_problem()
    n = op.n
    assert solve.objective(op, y, np.zeros((n, n), complex), lam, levels, "haar") == pytest.approx(
        np.vdot(y, y).real, rel=1e-14)
    assert _minimiser_holds(solve.objective, op, y, lam, levels, x_hat, f_min)

    def half_data(op, y, xp, lam, levels, wname):
        r = op.A(solve.crop(xp, op.n)) - y
        w = wavelet.dwt2(xp, levels, wname)
        det = wavelet.detail_mask(*xp.shape[-2:], levels)
        return 0.5 * np.vdot(r, r).real + lam * np.sum(np.abs(w[det]))

    def ll_penalised(op, y, xp, lam, levels, wname):
        r = op.A(solve.crop(xp, op.n)) - y
        return np.vdot(r, r).real + lam * np.sum(np.abs(wavelet.dwt2(xp, levels, wname)))

    def squared_l1(op, y, xp, lam, levels, wname):
        r = op.A(solve.crop(xp, op.n)) - y
        w = wavelet.dwt2(xp, levels, wname)
        det = wavelet.detail_mask(*xp.shape[-2:], levels)
        return np.vdot(r, r).real + lam * np.sum(np.abs(w[det]) ** 2)

    for mutant in (half_data, ll_penalised, squared_l1):
        assert not _minimiser_holds(mutant, op, y, lam, levels, x_hat, f_min), mutant.__name__
    # the minimiser check alone (value pin aside) also sees the first two mistakes
    for mutant in (half_data, ll_penalised):
        f_mut = mutant(op, y, x_hat, lam, levels, "haar")
        assert not _minimiser_holds(mutant, op, y, lam, levels, x_hat, f_mut), mutant.__name__


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
