"""Failure reporting of the solvers (expenc_solve_status) and the per-problem
scalars of calls with more than one workgroup's worth of problems.

* a NaN placed in the measured data y (plain data: the kernels only compute
  with it) must come back as EXPENC_ENONFINITE from FISTA (FP32 and fp16
  split), CG and a batched solve; a healthy solve reports EXPENC_OK;
* FISTA with the objective trace on and a step 1/L eight times too long
  (L underestimated) diverges: EXPENC_EDIVERGED, while the same solve with
  the correct L stays below F(0) = ||y||^2 at every iteration;
* pre-whitening with a noise covariance that is not positive definite
  reports EXPENC_ENONFINITE;
* 300 same-geometry problems in one batched call (more than the 256 threads
  of one workgroup) against single solves on the same inputs, with L given
  and from the power iteration; CG with 300 right-hand sides of one operator
  against the FP64 oracle's CG, column by column."""
import numpy as np
import pytest

import synth
from oracle import solve
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu


def _ee():
    import paper_2211_07532_amd as ee
    return ee


def _tiny():
    w = synth.TINY
    c = Case(w, sh=True)
    op = solve.Operator(c.smaps, c.coef, c.time, c.basis_np, c.dw0, w.n)
    y = c64(op.A(c.x_noisy))
    L = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 7)), 20)
    lam = solve.lambda_rule(op, y)
    return w, c, op, y, L, lam


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_fista_nan_in_data_is_reported(prec):
    ee = _ee()
    from paper_2211_07532_amd import _binding as b
    w, c, op, y, L, lam = _tiny()
    ok = ee.fista(c.to_dev(y), c.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam,
                  check_status=False)
    assert ok.status == b.EXPENC_OK
    bad = y.copy()
    bad[100, 3] = np.nan
    print(f"[case] FISTA {prec} with one NaN sample", flush=True)
    res = ee.fista(c.to_dev(bad), c.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam,
                   check_status=False)
    assert res.status == b.EXPENC_ENONFINITE
    with pytest.raises(b.ExpencError) as ei:
        ee.fista(c.to_dev(bad), c.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam)
    assert ei.value.status == b.EXPENC_ENONFINITE
    # the status is per call: the next healthy solve on the same workspace is clean again
    again = ee.fista(c.to_dev(y), c.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam,
                     check_status=False)
    assert again.status == b.EXPENC_OK


def test_fista_divergence_is_reported():
    ee = _ee()
    from paper_2211_07532_amd import _binding as b
    w, c, op, y, L, lam = _tiny()
    good = ee.fista(c.to_dev(y), c.op, w.n_iter, w.levels, w.wavelet, lipschitz=L, lam=lam, trace=True,
                    check_status=False)
    f0 = float(np.vdot(y, y).real)
    obj = good.objective.cpu().numpy()[0]
    print(f"[case] healthy trace max F {obj.max():.4e} vs F(0) {f0:.4e}", flush=True)
    assert good.status == b.EXPENC_OK and np.all(obj <= f0)
    # step 8/L: the top eigen-direction grows by |1 - 8| per iteration
    res = ee.fista(c.to_dev(y), c.op, 12, w.levels, w.wavelet, lipschitz=L / 8, lam=lam, trace=True,
                   check_status=False)
    obj = res.objective.cpu().numpy()[0]
    print(f"[case] L/8 trace: last F {obj[-1]:.4e}", flush=True)
    assert np.all(np.isfinite(obj)) and obj[-1] > f0
    assert res.status == b.EXPENC_EDIVERGED
    with pytest.raises(b.ExpencError) as ei:
        ee.fista(c.to_dev(y), c.op, 12, w.levels, w.wavelet, lipschitz=L / 8, lam=lam, trace=True)
    assert ei.value.status == b.EXPENC_EDIVERGED


def test_cg_and_batched_nan_are_reported():
    ee = _ee()
    from paper_2211_07532_amd import _binding as b
    w, c, op, y, L, lam = _tiny()
    bad = y.copy()
    bad[7, 0] = np.nan
    ee.cg(c.to_dev(y), c.op, 5, check_status=True)  # healthy: no exception
    with pytest.raises(b.ExpencError) as ei:
        ee.cg(c.to_dev(bad), c.op, 5, check_status=True)
    assert ei.value.status == b.EXPENC_ENONFINITE
    ys = [c.to_dev(y), c.to_dev(bad)]
    ee.fista_batched([ys[0], ys[0]], [c.op, c.op], 5, w.levels, w.wavelet, lipschitz=L, lam=lam, check_status=True)
    with pytest.raises(b.ExpencError) as ei:
        ee.fista_batched(ys, [c.op, c.op], 5, w.levels, w.wavelet, lipschitz=L, lam=lam, check_status=True)
    assert ei.value.status == b.EXPENC_ENONFINITE


def test_prewhiten_non_pd_covariance_is_reported():
    import torch
    ee = _ee()
    from paper_2211_07532_amd import _binding as b
    C = 4
    rng = np.random.default_rng(3)
    y = torch.from_numpy((rng.standard_normal((64, C)) + 1j * rng.standard_normal((64, C))).astype(np.complex64))
    psi = np.eye(C, dtype=np.complex128)
    ee.prewhiten(torch.from_numpy(psi).cuda(), y.clone().cuda())  # positive definite: no exception
    psi[2, 2] = -1.0
    with pytest.raises(b.ExpencError) as ei:
        ee.prewhiten(torch.from_numpy(psi).cuda(), y.clone().cuda())
    assert ei.value.status == b.EXPENC_ENONFINITE


def _small_same_shape(nprob, n=8, ncoils=2, nsamples=96, n_iter=4):
    out = []
    for k in range(nprob):
        out.append(synth.Workload(f"many-{k}", n, 0.222, ncoils, nsamples, 2e-6, 2.0, 4, 50.0, 20.0, n_iter, "haar",
                                  1, 2000 + k))
    return out


@pytest.mark.parametrize("given_L", [True, False], ids=["L-given", "L-power"])
def test_batched_more_than_256_problems(given_L):
    ee = _ee()
    ws = _small_same_shape(300)
    cases = [Case(wk, sh=True) for wk in ws]
    ops = [solve.Operator(ca.smaps, ca.coef, ca.time, ca.basis_np, ca.dw0, wk.n) for ca, wk in zip(cases, ws)]
    ys = [c64(o.A(ca.x_noisy)) for o, ca in zip(ops, cases)]
    v0 = c64(synth.power_start(ws[0].npix, 5))
    L = 0.0
    if given_L:
        L = 1.5 * max(solve.power_lipschitz(o, v0, 20) for o in ops[:4])
    print(f"[case] 300 problems of 8x8 in one batched call, L given: {given_L}", flush=True)
    xs = ee.fista_batched([ca.to_dev(y) for ca, y in zip(cases, ys)], [ca.op for ca in cases], ws[0].n_iter,
                          ws[0].levels, "haar", lipschitz=L, power_v0=cases[0].to_dev(v0), n_power=10, lam=-1.0,
                          lambda_factor=1e-3, check_status=True)
    for k in (0, 1, 255, 256, 257, 299):
        single = ee.fista(cases[k].to_dev(ys[k]), cases[k].op, ws[k].n_iter, ws[k].levels, "haar", lipschitz=L,
                          power_v0=cases[k].to_dev(v0), n_power=10, lam=-1.0, lambda_factor=1e-3)
        e = rel(xs[k].cpu().numpy(), single.x.cpu().numpy())
        print(f"  problem {k}: batched vs single {e:.2e}", flush=True)
        assert np.all(np.isfinite(xs[k].cpu().numpy())) and e <= 1e-5


def test_cg_300_right_hand_sides_match_oracle():
    ee = _ee()
    w = synth.Workload("cg-many", 12, 0.222, 1, 300, 2e-6, 1.5, 4, 50.0, 20.0, 3, "haar", 1, 77)
    c = Case(w, sh=True)
    op = solve.Operator(c.smaps, c.coef, c.time, c.basis_np, c.dw0, w.n)
    rng = np.random.default_rng(9)
    xs = c64(rng.standard_normal((300, w.npix)) + 1j * rng.standard_normal((300, w.npix)))
    ys = np.stack([c64(op.A(x)) for x in xs])          # [300][T][1]
    print("[case] CG, 1 coil, 300 right-hand sides, 3 iterations", flush=True)
    got = ee.cg(c.to_dev(ys), c.op, 3, check_status=True).cpu().numpy()
    for k in (0, 255, 256, 299):
        ref = solve.cg_ls(op, ys[k], 3)
        e = rel(got[k], ref)
        print(f"  column {k}: rel {e:.2e}", flush=True)
        assert e <= 1e-5
