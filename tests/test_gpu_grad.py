"""GPU parity of the differentiation path: the field-gradient kernel against
the oracle's VJPs, the autograd Functions, the soft-threshold VJP, and an
unrolled FISTA (with and without per-iteration checkpointing) against the
FP64 oracle's autograd gradients.  Bars: 1e-4 relative for single-operator
gradients (FP32 operators, FP64 sums); 1e-3 (median over components kinds)
for the unrolled solve, where soft-threshold kinks amplify rounding."""
import numpy as np
import pytest

import synth
from oracle import encoding, solve, unrolled, wavelet
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu


def _ee():
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import autograd as ag
    return ee, ag


@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_field_grad_matches_oracle_vjps(name, sh):
    ee, ag = _ee()
    if name == "tiny":
        w = synth.TINY
        case = Case(w, sh=sh)
    else:
        w = synth.Workload("ragged", 13, 0.1, 5, 333, 3e-6, 2.0, 16, 120.0, 20.0, 5, "haar", 1, 21)
        case = Case(w, z0=0.004, sh=sh)
    args = case.oracle_args()
    x = case.x_noisy
    g = c64(synth.random_complex((w.nsamples, case.smaps.shape[0]), 71))
    _, gc_ref, gd_ref = encoding.vjp_forward(x, g, *args)
    gc, gd = ag.field_grad(case.op, case.to_dev(x), case.to_dev(g))
    e1, e2 = rel(gc.cpu().numpy(), gc_ref), rel(gd.cpu().numpy(), gd_ref)
    gx = c64(synth.random_complex(w.npix, 72))
    y = c64(synth.random_complex((w.nsamples, case.smaps.shape[0]), 73))
    _, gc2_ref, gd2_ref = encoding.vjp_adjoint(y, gx, *args)
    gc2, gd2 = ag.field_grad(case.op, case.to_dev(gx), case.to_dev(y))
    e3, e4 = rel(gc2.cpu().numpy(), gc2_ref), rel(gd2.cpu().numpy(), gd2_ref)
    print(f"field grad {name} sh={sh}: fwd coef {e1:.2e} dw0 {e2:.2e}; adj coef {e3:.2e} dw0 {e4:.2e}", flush=True)
    assert max(e1, e2, e3, e4) <= 1e-4


@pytest.mark.parametrize("mode", ["forward", "adjoint"])
def test_field_grad_full_size_diff_config(mode):
    """The differentiation workload's operator (128 x 128, 16 coils, T = 12000,
    16 field terms + dB0, solid-harmonic kind) at full size against the
    oracle's VJPs of the forward and of the adjoint operator."""
    ee, ag = _ee()
    w = synth.DIFF
    case = Case(w, sh=True)
    args = case.oracle_args()
    print(f"[case] field grad full {w.name} {mode}", flush=True)
    if mode == "forward":
        x = case.x_noisy
        g = c64(synth.random_complex((w.nsamples, w.ncoils), 81))
        _, gc_ref, gd_ref = encoding.vjp_forward(x, g, *args)
        gc, gd = ag.field_grad(case.op, case.to_dev(x), case.to_dev(g))
    else:
        gx = c64(synth.random_complex(w.npix, 82))
        y = c64(synth.random_complex((w.nsamples, w.ncoils), 83))
        _, gc_ref, gd_ref = encoding.vjp_adjoint(y, gx, *args)
        gc, gd = ag.field_grad(case.op, case.to_dev(gx), case.to_dev(y))
    e1, e2 = rel(gc.cpu().numpy(), gc_ref), rel(gd.cpu().numpy(), gd_ref)
    print(f"  coef {e1:.2e}  dw0 {e2:.2e}", flush=True)
    assert max(e1, e2) <= 1e-4


def test_unrolled_full_size_checkpointing_is_exact():
    """10 unrolled iterations on the full differentiation workload: the
    checkpointed backward reproduces the stored-iterate gradients bit for bit
    (the FP64 oracle of the unrolled solve is checked at a smaller size)."""
    import torch
    ee, ag = _ee()
    w = synth.DIFF
    case = Case(w, z0=0.0)
    L = 1.01 * float(ee.lipschitz(case.op, case.to_dev(c64(synth.power_start(w.npix, 9))), 30))
    y0 = ee.forward(case.to_dev(case.x_noisy), case.op)
    lam = 1e-3 * float(torch.max(torch.abs(ee.adjoint(y0, case.op))))
    print(f"[case] unrolled full {w.name}: L {L:.4e} lambda {lam:.4e}", flush=True)
    l1, gx1, gc1, gd1 = _gpu_unrolled(ag, w, case, L, lam, ckpt=True)
    l0, gx0, gc0, gd0 = _gpu_unrolled(ag, w, case, L, lam, ckpt=False)
    assert np.isfinite(l1) and l0 == l1
    assert np.array_equal(gx0.view(np.uint32), gx1.view(np.uint32))
    assert np.array_equal(gc0, gc1) and np.array_equal(gd0, gd1)
    assert np.linalg.norm(gc1) > 0 and np.linalg.norm(gd1) > 0


def test_autograd_functions_match_oracle():
    import torch
    ee, ag = _ee()
    w = synth.TINY
    case = Case(w)
    spec = ag.OperatorSpec(w.n, w.n, case.t_smaps, case.t_time, basis=case.t_basis)
    x = case.to_dev(case.x_noisy).reshape(1, -1).requires_grad_(True)
    coef = case.t_coef.clone().requires_grad_(True)
    dw0 = case.t_dw0.clone().requires_grad_(True)
    g = c64(synth.random_complex((1, w.nsamples, w.ncoils), 74))
    y = ag.ExpEncForward.apply(x, coef, dw0, spec)
    # loss = Re <g, y>  =>  dL/dy = g
    loss = torch.sum((torch.from_numpy(g.astype(np.complex64)).cuda().conj() * y).real)
    loss.backward()
    gx_ref, gc_ref, gd_ref = encoding.vjp_forward(case.x_noisy, g[0], *case.oracle_args())
    assert rel(x.grad.cpu().numpy()[0], gx_ref) <= 1e-5
    assert rel(coef.grad.cpu().numpy(), gc_ref) <= 1e-4
    assert rel(dw0.grad.cpu().numpy(), gd_ref) <= 1e-4
    # adjoint Function
    yy = torch.from_numpy(g.astype(np.complex64)).cuda().requires_grad_(True)
    coef2 = case.t_coef.clone().requires_grad_(True)
    dw02 = case.t_dw0.clone().requires_grad_(True)
    gxv = c64(synth.random_complex((1, w.npix), 75))
    xo = ag.ExpEncAdjoint.apply(yy, coef2, dw02, spec)
    torch.sum((torch.from_numpy(gxv.astype(np.complex64)).cuda().conj() * xo).real).backward()
    gy_ref, gc2_ref, gd2_ref = encoding.vjp_adjoint(g[0], gxv[0], *case.oracle_args())
    assert rel(yy.grad.cpu().numpy()[0], gy_ref) <= 1e-5
    assert rel(coef2.grad.cpu().numpy(), gc2_ref) <= 1e-4
    assert rel(dw02.grad.cpu().numpy(), gd2_ref) <= 1e-4


def test_soft_threshold_vjp_matches_oracle_autograd():
    import torch
    ee, ag = _ee()
    wv = c64(synth.random_complex((32, 32), 76))
    g = c64(synth.random_complex((32, 32), 77))
    tau = 0.9
    wt = torch.from_numpy(wv).requires_grad_(True)
    out = unrolled.soft(wt, tau, 2)
    torch.sum((torch.from_numpy(g).conj() * out).real).backward()
    ref = wt.grad.numpy()
    wd = torch.from_numpy(wv.astype(np.complex64)).cuda().requires_grad_(True)
    o = ag.SoftThreshold.apply(wd, tau, 2)
    torch.sum((torch.from_numpy(g.astype(np.complex64)).cuda().conj() * o).real).backward()
    assert rel(wd.grad.cpu().numpy(), ref) <= 1e-6


def _unrolled_case(n=16, c=4, t=400, n_iter=5, wname="db4", levels=2, seed=81):
    w = synth.Workload("unr", n, 0.2, c, t, 4e-6, 2.0, 16, 80.0, 15.0, n_iter, wname, levels, seed)
    case = Case(w, z0=0.003)
    op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, n)
    L = 1.01 * solve.power_lipschitz(op, c64(synth.power_start(w.npix, 2)), 60)
    lam = solve.lambda_rule(op, op.A(case.x_noisy), 0.02)
    return w, case, L, lam


def _gpu_unrolled(ag, w, case, L, lam, ckpt):
    import torch
    spec = ag.OperatorSpec(w.n, w.n, case.t_smaps, case.t_time, basis=case.t_basis)
    x_in = case.to_dev(case.x_noisy).reshape(1, -1).requires_grad_(True)
    coef = case.t_coef.clone().requires_grad_(True)
    dw0 = case.t_dw0.clone().requires_grad_(True)
    y = ag.ExpEncForward.apply(x_in, coef, dw0, spec)
    xh = ag.unrolled_fista(y, coef, dw0, spec, L, lam, w.n_iter, w.levels, w.wavelet, use_checkpoint=ckpt)
    xt = case.to_dev(case.x_true).reshape(1, w.n, w.n)
    loss = torch.sum(torch.abs(xh - xt) ** 2)
    loss.backward()
    return (loss.item(), x_in.grad.cpu().numpy()[0], coef.grad.cpu().numpy(), dw0.grad.cpu().numpy())


def test_unrolled_fista_gradients_and_checkpointing():
    ee, ag = _ee()
    w, case, L, lam = _unrolled_case()
    loss_ref, gx_ref, gc_ref, gd_ref = unrolled.loss_and_grads(case.x_noisy, case.x_true, case.smaps, case.coef,
                                                               case.time, case.basis_np, case.dw0, L, lam, w.n_iter,
                                                               w.levels, w.wavelet, w.n, w.n_pad)
    l1, gx1, gc1, gd1 = _gpu_unrolled(ag, w, case, L, lam, ckpt=True)
    l0, gx0, gc0, gd0 = _gpu_unrolled(ag, w, case, L, lam, ckpt=False)
    errs = [rel(gx1, gx_ref), rel(gc1, gc_ref), rel(gd1, gd_ref)]
    print(f"unrolled: loss {l1:.6e} vs {loss_ref:.6e}; grad errors x {errs[0]:.2e} coef {errs[1]:.2e} "
          f"dw0 {errs[2]:.2e}", flush=True)
    assert abs(l1 - loss_ref) <= 1e-4 * loss_ref
    assert max(errs) <= 1e-3
    # checkpointed recomputation reproduces the stored-iterate gradients bit for bit
    assert l0 == l1
    assert np.array_equal(gx0.view(np.uint32), gx1.view(np.uint32))
    assert np.array_equal(gc0, gc1) and np.array_equal(gd0, gd1)


GOLDEN_DIFF = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "diff_unrolled.npz")


def test_unrolled_gradients_match_fp64_oracle_at_diff_config():
    """The differentiation workload at full size (128 x 128, 16 coils,
    T = 12000, 16 field terms + dB0, 10 unrolled FISTA iterations, db4 J = 3):
    the loss and the checkpointed gradients with respect to x_in, k_l(t) and
    dB0 against the FP64 oracle's reverse pass (tests/golden/diff_unrolled.npz,
    written by tests/golden/make_golden.py diff with the same L and lambda):
    loss within 1e-4, each gradient within 1e-3 (relative l2)."""
    import os
    if not os.path.exists(GOLDEN_DIFF):
        pytest.skip("golden file missing: run tests/golden/make_golden.py diff")
    ee, ag = _ee()
    g = np.load(GOLDEN_DIFF)
    w = synth.DIFF
    case = Case(w)
    L, lam = float(g["lipschitz"]), float(g["lam"])
    print(f"[case] unrolled gradients vs oracle, {w.name}: L {L:.4e} lambda {lam:.4e}", flush=True)
    loss, gx, gc, gd = _gpu_unrolled(ag, w, case, L, lam, ckpt=True)
    errs = {"x": rel(gx, g["grad_x"]), "coef": rel(gc, g["grad_coef"]), "dw0": rel(gd, g["grad_dw0"])}
    e_loss = abs(loss - float(g["loss"])) / float(g["loss"])
    print(f"  loss {loss:.6e} vs {float(g['loss']):.6e} ({e_loss:.2e}); gradient errors "
          + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert e_loss <= 1e-4
    assert max(errs.values()) <= 1e-3
