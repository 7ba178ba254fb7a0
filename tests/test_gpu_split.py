"""GPU parity of the split-precision (bf16 / fp16 hi+lo) operator forms and of
the anchored-refinement FISTA against the FP64 oracle.

Bars: relative l2 error of A / A^H <= 1e-3 in split form (the target for the
split operators before refinement), and, in both directions, no worse than
5x the error level the RNE split emulation predicts for the same arithmetic
(plus 2e-6 for the FP32 phase increments); image NRMSE after a split-form
solve <= 1e-4 under each anchor mode (FP32 at the ends and split
between, all FP32, all split after the first).  Whole-output full-size parity is in
test_gpu_fullsize.py.  The solid-harmonic adjoint forms its phase row by row
over 32-pixel blocks: the 13 px grid (rows padded to 16) has every block
continue into the next row, the 20 and 32 px grids (rows padded to 32) none,
and the 1.1 mm grid of the full-size tests some."""
import numpy as np
import pytest

import synth
from oracle import encoding, solve
from tests.gpu_common import Case, c64, emulated_split_errors, rel

pytestmark = pytest.mark.gpu


def _ee():
    import paper_2211_07532_amd as ee
    return ee


@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("name", ["tiny", "ragged", "40coils-nodw0"])
def test_split_operators(prec, name, sh):
    ee = _ee()
    if name == "tiny":
        w = synth.TINY
        case = Case(w, sh=sh)
        batch = 2
    elif name == "ragged":
        w = synth.Workload("ragged", 13, 0.1, 5, 333, 3e-6, 2.0, 16, 120.0, 20.0, 5, "haar", 1, 21)
        case = Case(w, z0=0.004, sh=sh)
        batch = 3
    else:
        w = synth.Workload("c40", 20, 0.2, 40, 700, 2e-6, 2.0, 9, 80.0, 20.0, 5, "haar", 1, 23)
        case = Case(w, with_dw0=False, sh=sh)
        batch = 1
    print(f"[case] split {prec} {name} sh={sh}", flush=True)
    x = c64(synth.random_complex((batch, w.npix), 61))
    x[0] = case.x_noisy
    y_ref = encoding.forward(x, *case.oracle_args())
    y = ee.forward(case.to_dev(x), case.op, precision=prec).cpu().numpy()
    e_fwd = rel(y, y_ref)
    g = c64(synth.random_complex(y_ref.shape, 62))
    x_ref = encoding.adjoint(g, *case.oracle_args())
    e_adj = rel(ee.adjoint(case.to_dev(g), case.op, precision=prec).cpu().numpy(), x_ref)
    # the adjoint is held to the emulation of its first image alone
    e_adj0 = rel(ee.adjoint(case.to_dev(g[:1]), case.op, precision=prec).cpu().numpy()[0], x_ref[0])
    emu_f, emu_a = emulated_split_errors(case, case.x_noisy, g[0], np.arange(w.nsamples), np.arange(w.npix), prec)
    e_fwd0 = rel(y[0], y_ref[0])
    print(f"split {prec} {name} sh={sh}: forward {e_fwd:.2e} ({e_fwd0:.2e} image 0, emulated {emu_f:.2e}), "
          f"adjoint {e_adj:.2e} ({e_adj0:.2e} image 0, emulated {emu_a:.2e})", flush=True)
    assert e_fwd <= 1e-3 and e_adj <= 1e-3
    assert e_fwd0 <= 5 * emu_f + 2e-6
    assert e_adj0 <= 5 * emu_a + 2e-6


@pytest.mark.parametrize("anchor", ["ends", "fp32", "split"])
@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("variant", ["tiny", "padded-db4"])
def test_split_fista_with_anchors(prec, variant, sh, anchor):
    ee = _ee()
    if variant == "tiny":
        w = synth.TINY
    else:
        w = synth.Workload("pad", 20, 0.2, 6, 900, 3e-6, 2.0, 16, 80.0, 20.0, 30, "db4", 3, 51)
    case = Case(w, sh=sh)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    L = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 4)), 30)
    lam = solve.lambda_rule(op, y)
    ref = solve.fista(op, y, L, lam, w.n_iter, w.levels, w.wavelet, w.n_pad)
    res = ee.fista(case.to_dev(y), case.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam,
                   refine_every=10, anchor=anchor)
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), ref)
    # without intermediate anchors (only the first and the last iteration are exact)
    res0 = ee.fista(case.to_dev(y), case.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L, lam=lam,
                    refine_every=10 ** 6, anchor=anchor)
    e0 = solve.nrmse(res0.x.cpu().numpy().reshape(-1), ref)
    print(f"split FISTA {prec} {variant} sh={sh} anchor={anchor}: NRMSE {e:.2e} (anchored every 10), "
          f"{e0:.2e} (no intermediate anchor)", flush=True)
    assert e <= 1e-4


@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_split_operators_scale_invariant(prec, sh):
    """The split forms keep their accuracy on inputs of any magnitude: the
    fp16 halves alone would flush values below ~6e-8 to zero and overflow
    above 65504, so the fp16 form scales every operand by a power of two
    chosen on the device.  Inputs scaled by 1e-12 ... 1e6 (bf16 has the FP32
    exponent range) must meet the unscaled case's error level."""
    ee = _ee()
    w = synth.TINY
    case = Case(w, sh=sh)
    x0 = c64(synth.random_complex((2, w.npix), 63))
    x0[0] = case.x_noisy
    g0 = c64(synth.random_complex((2, w.nsamples, w.ncoils), 64))
    errs = {}
    for s in (1.0, 1e-12, 1e-4, 1e6):
        x = c64(x0 * s)
        g = c64(g0 * s)
        e_f = rel(ee.forward(case.to_dev(x), case.op, precision=prec).cpu().numpy(),
                  encoding.forward(x, *case.oracle_args()))
        e_a = rel(ee.adjoint(case.to_dev(g), case.op, precision=prec).cpu().numpy(),
                  encoding.adjoint(g, *case.oracle_args()))
        errs[s] = (e_f, e_a)
    print(f"split {prec} sh={sh} errors by input scale: {errs}", flush=True)
    e1f, e1a = errs[1.0]
    for s, (e_f, e_a) in errs.items():
        assert e_f <= 3 * e1f + 1e-6 and e_a <= 3 * e1a + 1e-6, s
    # all-zero inputs (a zero magnitude bound: unscaled) give exact zeros
    assert not ee.forward(case.to_dev(0 * x0), case.op, precision=prec).cpu().numpy().any()
    assert not ee.adjoint(case.to_dev(0 * g0), case.op, precision=prec).cpu().numpy().any()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_split_fista_on_scaled_data(prec):
    """The anchored split FISTA is equivariant in the data scale: with y and
    lambda scaled by s the solution scales by s.  Data scaled by 2^-23 and
    2^17 (outside the fp16 range either way) against the oracle's unscaled
    solve."""
    ee = _ee()
    w = synth.TINY
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    L = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 4)), 30)
    lam = solve.lambda_rule(op, y)
    ref = solve.fista(op, y, L, lam, w.n_iter, w.levels, w.wavelet, w.n_pad)
    for s in (2.0 ** -23, 2.0 ** 17):  # powers of two: the scaled data are exact
        res = ee.fista(case.to_dev(y * s), case.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=L,
                       lam=lam * s, refine_every=10)
        e = solve.nrmse(res.x.cpu().numpy().reshape(-1) / s, ref)
        print(f"split FISTA {prec} data scale {s:.1e}: NRMSE {e:.2e}", flush=True)
        assert e <= 1e-4, s


@pytest.mark.parametrize("n", [32, 13], ids=["rows-aligned", "rows-crossing"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_strong_field_operators(prec, n):
    """Fields far beyond the paper's (every field term x30 and the off-
    resonance map x10: up to 63 (13 px) and 357 (32 px) turns of phase
    within one 32-sample tile, 14-16 turns between neighbouring pixels)
    stay accurate: the phase is reduced to turns before every sine and
    cosine, and the FP32 increments of the split forms stay small against
    their tiles.  Measured: split forms 0.4-2.2e-5 (held to 1e-4, a tenth of
    the split operators' bar), FP32 1.2e-7 (held to 1e-6; its phase is FP64
    per entry).  Grids of 32 px and 13 px take the adjoint's
    two kernel variants (32-pixel blocks inside image rows / continuing into
    the next row)."""
    import torch
    ee = _ee()
    w = synth.Workload("strong", n, 0.1, 6, 700, 3e-6, 2.0, 16, 100.0, 20.0, 5, "haar", 1, 71)
    case = Case(w, sh=True)
    coef, dw0 = case.coef * 30.0, case.dw0 * 10.0
    dev = torch.device("cuda")
    op = ee.Operator(n, n, case.t_smaps, torch.from_numpy(coef).to(dev), case.t_time, None,
                     torch.from_numpy(dw0).to(dev), sh_grid=(w.fov, w.fov, case.z0))
    args = (case.smaps, coef, case.time, case.basis_np, dw0)
    phi = encoding.phase(coef, case.time, case.basis_np, dw0) / (2 * np.pi)
    print(f"[case] strong field {prec} n={n}: phase spans {np.ptp(phi):.0f} turns, "
          f"{np.abs(np.diff(phi, axis=0)).max():.2f} turns per sample", flush=True)
    x = c64(synth.random_complex((2, w.npix), 72))
    g = c64(synth.random_complex((2, w.nsamples, w.ncoils), 73))
    e_f = rel(ee.forward(case.to_dev(x), op, precision=prec).cpu().numpy(), encoding.forward(x, *args))
    e_a = rel(ee.adjoint(case.to_dev(g), op, precision=prec).cpu().numpy(), encoding.adjoint(g, *args))
    print(f"strong field {prec} n={n}: forward {e_f:.2e}, adjoint {e_a:.2e}", flush=True)
    bar = 1e-6 if prec == "fp32" else 1e-4
    assert e_f <= bar and e_a <= bar
