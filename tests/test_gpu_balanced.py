"""GPU parity of the paper's regulariser against the FP64 oracle: the
undecimated wavelet transform and its adjoint (Haar and db4, 1-3 levels,
odd, even and non-square grids, batches), the sigma/2 weight rule (exact
histogram counts on identical coefficients), and balanced FISTA (L_A and the
oracle's weights given, kappa = L_A; the device's own weight rule, which
starts from its FP32 A^H y, within one histogram bin of the oracle's).
Bars: 1e-6 (transform), 1e-12 relative (weights on identical coefficients),
NRMSE 1e-5 (FP32 solve) / 1e-4 (split)."""
import numpy as np
import pytest

import synth
from oracle import balanced as bal
from oracle import solve
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu


def _dev(a, dtype=np.complex64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


@pytest.mark.parametrize("name", ["haar", "db4"])
@pytest.mark.parametrize("shape,levels,batch", [((13, 13), 1, 1), ((16, 20), 2, 2), ((32, 32), 3, 1),
                                                ((152, 148), 1, 1)])
def test_undecimated_transform_matches_oracle(name, shape, levels, batch):
    import paper_2211_07532_amd as ee
    rng = np.random.default_rng(sum(shape) + levels)
    x = c64(rng.standard_normal((batch,) + shape) + 1j * rng.standard_normal((batch,) + shape))
    ref = np.stack([bal.swt2(x[b], levels, name) for b in range(batch)])
    w = ee.swt_fwd(_dev(x), levels, name)
    e1 = rel(w.cpu().numpy(), ref)
    v = c64(rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape))
    ref2 = np.stack([bal.iswt2(v[b], levels, name) for b in range(batch)])
    e2 = rel(ee.swt_inv(_dev(v), levels, name).cpu().numpy(), ref2)
    e3 = rel(ee.swt_inv(w, levels, name).cpu().numpy(), x)
    print(f"[case] swt {name} {shape} J={levels} B={batch}: fwd {e1:.2e} adj {e2:.2e} inv(fwd) {e3:.2e}", flush=True)
    assert max(e1, e2, e3) <= 1e-6


@pytest.mark.parametrize("levels", [1, 2])
def test_sigma_weights_match_oracle(levels):
    import paper_2211_07532_amd as ee
    w = synth.TINY
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    coefs = c64(bal.swt2(op.AH(y).reshape(w.n, w.n), levels, "db4"))
    lam_ref = bal.sigma_weights(coefs, levels)
    lam, counts = ee.sigma_weights(_dev(coefs[None]), levels, counts=True)
    lam = lam.cpu().numpy()[0]
    counts = counts.cpu().numpy()[0]
    for j in range(levels):
        m = np.abs(coefs[3 * j:3 * j + 3]).ravel()
        width = 4.0 * np.mean(m) / 256
        idx = np.floor(m / width).astype(np.int64)
        ref_counts = np.bincount(idx[idx < 256], minlength=256)
        moved = int(np.sum(np.abs(counts[j] - ref_counts)))
        print(f"[case] sigma weights J={levels} level {j}: lambda {lam[3 * j]:.6e} (ref {lam_ref[3 * j]:.6e}), "
              f"counts moved {moved}", flush=True)
        assert moved <= 2
    assert lam[-1] == 0.0
    assert np.max(np.abs(lam - lam_ref)) <= 1e-12 * np.max(lam_ref)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("name,levels", [("db4", 1), ("haar", 2)])
def test_balanced_fista_matches_oracle(prec, name, levels):
    import paper_2211_07532_amd as ee
    w = synth.Workload("bal", 20, 0.2, 6, 900, 3e-6, 2.0, 16, 80.0, 20.0, 12, name, levels, 71)
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    L_A = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 3)), 30)
    lam = bal.sigma_weights(bal.swt2(op.AH(y).reshape(w.n, w.n), levels, name), levels)
    ref = bal.fista(op, y, L_A, L_A, lam, w.n_iter, levels, name)
    # the solve with the oracle's weights passed in
    import torch
    res = ee.fista_balanced(case.to_dev(y), case.op, w.n_iter, levels, name, precision=prec, lipschitz=L_A,
                            lam=torch.from_numpy(lam).cuda())
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), ref.reshape(-1))
    # the device's own sigma/2 rule (FP32 A^H y): the same histogram bin, or a neighbour
    res2 = ee.fista_balanced(case.to_dev(y), case.op, 0, levels, name, lipschitz=L_A)
    coefs = bal.swt2(op.AH(y).reshape(w.n, w.n), levels, name)
    width = np.array([4.0 * np.mean(np.abs(coefs[3 * j:3 * j + 3])) / 256 for j in range(levels)])
    el = np.max([abs(res2.lam.numpy()[0][3 * j] - lam[3 * j]) / (0.5 * width[j]) for j in range(levels)])
    print(f"[case] balanced {prec} {name} J={levels}: NRMSE {e:.2e}, device weights within {el:.2f} bins, "
          f"kappa {res.kappa:.4e}", flush=True)
    assert abs(res.kappa - L_A) <= 1e-12 * L_A and abs(res.lipschitz_a - L_A) <= 1e-12 * L_A
    assert el <= 1.0 + 1e-6
    assert e <= (1e-5 if prec == "fp32" else 1e-4)


@pytest.mark.parametrize("anchor", ["ends", "fp32", "split"])
def test_balanced_fista_anchor_modes_match_oracle(anchor):
    """The balanced solver's split form (fp16) under each anchor mode against
    the FP64 oracle's balanced FISTA, with the oracle's weights passed in."""
    import paper_2211_07532_amd as ee
    import torch
    w = synth.Workload("bal", 20, 0.2, 6, 900, 3e-6, 2.0, 16, 80.0, 20.0, 12, "db4", 1, 71)
    case = Case(w, sh=True)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
    y = c64(op.A(case.x_noisy))
    L_A = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 3)), 30)
    lam = bal.sigma_weights(bal.swt2(op.AH(y).reshape(w.n, w.n), 1, "db4"), 1)
    ref = bal.fista(op, y, L_A, L_A, lam, w.n_iter, 1, "db4")
    res = ee.fista_balanced(case.to_dev(y), case.op, w.n_iter, 1, "db4", precision="fp16", lipschitz=L_A,
                            lam=torch.from_numpy(lam).cuda(), refine_every=4, anchor=anchor)
    e = solve.nrmse(res.x.cpu().numpy().reshape(-1), ref.reshape(-1))
    print(f"[case] balanced fp16 anchor={anchor}: NRMSE {e:.2e}", flush=True)
    assert e <= 1e-4
