"""Whole-output parity of A and A^H at the full 1.5 mm (148^2, 32 coils,
T = 16384) and 1.1 mm (200^2, 32 coils, T = 40000) sizes, in every form
(FP32, bf16 split, fp16 split) and both basis kinds (maps given as data,
solid harmonics evaluated by the library), in the benchmark's launch shapes,
against the FP64 oracle's whole outputs (eq. 1's operator and its adjoint).

Bars, per direction:
* FP32: relative l2 error <= 1e-5 and max|out - ref| <= 1e-5 max|ref|;
* split forms: relative l2 error <= 1e-3, and <= 5x the error that the
  round-to-nearest-even emulation of the same three-product arithmetic
  (phase tile rounded to FP32, then split) shows on the same problem --
  its error energy estimated from 64 uniformly drawn output rows (forward)
  / pixels (adjoint), normalised by the whole output's exact norm -- plus
  2e-6 for the FP32 phase increments; max|out - ref| <= the same level
  times max|ref|.
The oracle's outputs are computed once per size (module fixture)."""
import numpy as np
import pytest

import synth
from oracle import encoding
from tests.gpu_common import Case, c64, emulated_split_errors, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[synth.MM15, synth.MM11], ids=["1.5mm", "1.1mm"])
def full(request):
    wl = request.param
    print(f"[case] oracle outputs at {wl.name}", flush=True)
    cases = {False: Case(wl, sh=False), True: Case(wl, sh=True)}
    c = cases[True]
    x = c.x_noisy
    y_ref = encoding.forward(x, *c.oracle_args())
    g = c64(y_ref)                       # the adjoint's input: the data, rounded to complex64
    x_ref = encoding.adjoint(g, *c.oracle_args())
    # 64 uniformly drawn rows / pixels estimate the error energy of the whole
    # output, normalised by its exact norm
    rng = np.random.default_rng(17)
    ts = np.sort(rng.choice(wl.nsamples, 64, replace=False))
    rs = np.sort(rng.choice(wl.npix, 64, replace=False))
    emu = {k: emulated_split_errors(c, x, g, ts, rs, k, np.linalg.norm(y_ref), np.linalg.norm(x_ref))
           for k in ("bf16", "fp16")}
    print(f"  emulated split errors (forward, adjoint): {emu}", flush=True)
    return wl, cases, x, y_ref, g, x_ref, emu


@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_full_size_whole_outputs(full, prec, sh):
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import autotune
    wl, cases, x, y_ref, g, x_ref, emu = full
    case = cases[sh]
    autotune.apply_cached(case.op, 1, prec)      # the shipped launch shapes (the bench's)
    print(f"[case] whole outputs {wl.name} {prec} sh={sh}", flush=True)
    y = ee.forward(case.to_dev(x), case.op, precision=prec).cpu().numpy()
    xa = ee.adjoint(case.to_dev(g), case.op, precision=prec).cpu().numpy()
    e_f, e_a = rel(y, y_ref), rel(xa, x_ref)
    m_f = float(np.max(np.abs(y - y_ref)) / np.max(np.abs(y_ref)))
    m_a = float(np.max(np.abs(xa - x_ref)) / np.max(np.abs(x_ref)))
    print(f"  {wl.name} {prec} sh={sh}: forward l2 {e_f:.2e} max {m_f:.2e}, adjoint l2 {e_a:.2e} max {m_a:.2e}",
          flush=True)
    if prec == "fp32":
        bar_f = bar_a = 1e-5
    else:
        bar_f = min(1e-3, 5 * emu[prec][0] + 2e-6)
        bar_a = min(1e-3, 5 * emu[prec][1] + 2e-6)
    assert e_f <= bar_f and m_f <= bar_f
    assert e_a <= bar_a and m_a <= bar_a
    # adjoint identity on the GPU results (FP64 inner products)
    lhs = np.vdot(g.astype(np.complex128), y.astype(np.complex128))
    rhs = np.vdot(xa.astype(np.complex128), x)
    assert abs(lhs - rhs) / (np.linalg.norm(g) * np.linalg.norm(y)) <= max(bar_f, bar_a)
