"""Full-size solve parity: the 1.5 mm workload (148 x 148, 32 coils,
T = 16384, 16 field terms + dB0, 50 FISTA iterations, db4 J = 3) on the GPU
against the FP64 oracle's reconstruction stored in tests/golden/mm15_fista.npz
(written by tests/golden/make_golden.py, which calls only the oracle), and
the balanced-FISTA solve with the paper's regulariser against mm15_balanced.npz,
and the 1.1 mm workload (200 x 200, T = 40000, 100 iterations, db4 J = 4)
against mm11_fista.npz.
Bars: NRMSE <= 1e-5 in every form (the split forms with their default FP32
anchor cadences); L and lambda from the device rules within 1e-5."""
import os

import numpy as np
import pytest

import synth
from oracle import encoding, solve
from tests.gpu_common import Case, c64

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mm15_fista.npz")


@pytest.fixture(scope="module")
def mm15():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    g = np.load(GOLDEN)
    w = synth.MM15
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    return w, case, y, g


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_full_size_fista_matches_golden(mm15, prec):
    import paper_2211_07532_amd as ee
    w, case, y, g = mm15
    v0 = case.to_dev(c64(synth.power_start(w.npix, int(g["power_seed"]))))
    res = ee.fista(case.to_dev(y), case.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=0.0,
                   power_v0=v0, n_power=int(g["n_power"]), lam=-1.0, lambda_factor=1e-3)
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), g["x_hat"])
    print(f"golden {prec}: NRMSE {e:.2e}  L {res.lipschitz:.6e} (ref {float(g['lipschitz']):.6e})  "
          f"lambda {res.lam[0]:.6e} (ref {float(g['lam']):.6e})", flush=True)
    assert abs(res.lipschitz - float(g["lipschitz"])) <= 1e-5 * float(g["lipschitz"])
    assert abs(res.lam[0] - float(g["lam"])) <= 1e-5 * float(g["lam"])
    assert e <= 1e-5


@pytest.mark.parametrize("anchor", ["fp32", "ends"])
def test_full_size_fista_anchor_modes_match_golden(mm15, anchor):
    """The other two anchor modes of the split forms (every anchor in FP32
    at its cadence of 25; split anchors at 5 with the last one in FP32) on
    the full-size fp16 solve: both within 1e-5 of the FP64 solve."""
    import paper_2211_07532_amd as ee
    w, case, y, g = mm15
    v0 = case.to_dev(c64(synth.power_start(w.npix, int(g["power_seed"]))))
    res = ee.fista(case.to_dev(y), case.op, w.n_iter, w.levels, w.wavelet, precision="fp16", lipschitz=0.0,
                   power_v0=v0, n_power=int(g["n_power"]), lam=-1.0, lambda_factor=1e-3, anchor=anchor)
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), g["x_hat"])
    print(f"golden fp16 anchor={anchor}: NRMSE {e:.2e}", flush=True)
    assert e <= 1e-5


BALANCED = os.path.join(os.path.dirname(__file__), "golden", "mm15_balanced.npz")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_full_size_balanced_matches_golden(mm15, prec):
    """The paper's regulariser at full size: undecimated db4 (one level),
    sigma/2 weights, balanced FISTA with kappa = L_A, 50 iterations, against
    the FP64 oracle's solve in tests/golden/mm15_balanced.npz (L_A and the
    weights passed in).  The device's own weight rule (FP32 W A^H y) must land
    within one histogram bin of the oracle's."""
    import torch
    import paper_2211_07532_amd as ee
    from oracle import balanced as bal
    if not os.path.exists(BALANCED):
        pytest.skip("golden file missing: run tests/golden/make_golden.py balanced")
    w, case, y, _ = mm15
    g = np.load(BALANCED)
    L_A, levels, n_iter = float(g["lipschitz"]), int(g["levels"]), int(g["n_iter"])
    res = ee.fista_balanced(case.to_dev(y), case.op, n_iter, levels, "db4", precision=prec, lipschitz=L_A,
                            lam=torch.from_numpy(np.ascontiguousarray(g["lam"])).cuda())
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), g["x_hat"].reshape(-1))
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    coefs = bal.swt2(op.AH(y).reshape(w.n, w.n), levels, "db4")
    width = 4.0 * np.mean(np.abs(coefs[:3])) / 256
    dev = ee.fista_balanced(case.to_dev(y), case.op, 0, levels, "db4", lipschitz=L_A)
    dl = abs(dev.lam.numpy()[0][0] - float(g["lam"][0])) / (0.5 * width)
    print(f"golden balanced {prec}: NRMSE {e:.2e}, device sigma/2 weight within {dl:.2f} bins", flush=True)
    assert dl <= 1.0 + 1e-6
    assert e <= 1e-5


GOLDEN11 = os.path.join(os.path.dirname(__file__), "golden", "mm11_fista.npz")


@pytest.fixture(scope="module")
def mm11():
    if not os.path.exists(GOLDEN11):
        pytest.skip("golden file missing: run tests/golden/make_golden.py mm11")
    g = np.load(GOLDEN11)
    w = synth.MM11
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    return w, case, y, g


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_full_size_1p1mm_fista_matches_golden(mm11, prec):
    """The 1.1 mm configuration: FP32 against the split forms with FP32
    anchors, 100 iterations, final NRMSE against the FP64 oracle's solve
    (FP32 and fp16 within 1e-5; bf16, whose halves keep 16 bits, within the
    split forms' 1e-4)."""
    import paper_2211_07532_amd as ee
    w, case, y, g = mm11
    v0 = case.to_dev(c64(synth.power_start(w.npix, int(g["power_seed"]))))
    res = ee.fista(case.to_dev(y), case.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=0.0,
                   power_v0=v0, n_power=int(g["n_power"]), lam=-1.0, lambda_factor=1e-3)
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), g["x_hat"])
    print(f"golden 1.1 mm {prec}: NRMSE {e:.2e}  L {res.lipschitz:.6e} (ref {float(g['lipschitz']):.6e})  "
          f"lambda {res.lam[0]:.6e} (ref {float(g['lam']):.6e})", flush=True)
    assert abs(res.lipschitz - float(g["lipschitz"])) <= 1e-5 * float(g["lipschitz"])
    assert abs(res.lam[0] - float(g["lam"])) <= 1e-5 * float(g["lam"])
    assert e <= (1e-4 if prec == "bf16" else 1e-5)
