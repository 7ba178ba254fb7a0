"""GPU checks of the launch-shape autotuner: it picks one of its candidates
per direction, registers it (the plan the library reports changes
accordingly), caches it per device and geometry, and the operators stay
within the FP32 bar against the FP64 oracle under every tuned shape; a
batched solve planned with tuned totals matches the oracle."""
import numpy as np
import pytest

import synth
from oracle import encoding, solve
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu


def test_tune_registers_caches_and_keeps_parity(tmp_path):
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import autotune
    w = synth.Workload("tune", 40, 0.222, 8, 2400, 2e-6, 2.0, 16, 80.0, 20.0, 4, "db4", 2, 91, z0=0.002)
    case = Case(w, sh=True)
    cache = str(tmp_path / "tuning.json")
    cands = (256, 1024, 4096)
    try:
        for prec in ("fp32", "fp16"):
            default = autotune.plan_info(case.op, 1, prec)
            r = autotune.tune(case.op, 1, prec, candidates=cands, reps=3, path=cache, use_cache=False)
            print(f"[case] tune {prec}: fwd {r.fwd_target} ({r.fwd_ms:.4f} ms) adj {r.adj_target} "
                  f"({r.adj_ms:.4f} ms); default {default}", flush=True)
            assert r.fwd_target in cands and r.adj_target in cands and not r.cached
            info = autotune.plan_info(case.op, 1, prec)
            autotune.set_targets(case.op, 1, prec, r.fwd_target, r.adj_target)
            assert autotune.plan_info(case.op, 1, prec) == info
            # every candidate shape computes the same operator (to the FP32 / split bar)
            x = case.x_noisy
            y_ref = encoding.forward(x, *case.oracle_args())
            x_ref = encoding.adjoint(y_ref, *case.oracle_args())
            bar = 1e-5 if prec == "fp32" else 1e-3
            for t in cands:
                autotune.set_targets(case.op, 1, prec, t, t)
                y = ee.forward(case.to_dev(x), case.op, prec).cpu().numpy()
                xa = ee.adjoint(case.to_dev(c64(y_ref)), case.op, prec).cpu().numpy()
                assert rel(y.reshape(y_ref.shape), y_ref) <= bar
                assert rel(xa.reshape(x_ref.shape), x_ref) <= bar
            # the cache restores the tuned result in a later lookup
            autotune.set_targets(case.op, 1, prec, 0, 0)
            c = autotune.apply_cached(case.op, 1, prec, path=cache)
            assert c is not None and c.cached and (c.fwd_target, c.adj_target) == (r.fwd_target, r.adj_target)
            assert autotune.plan_info(case.op, 1, prec) == info
    finally:
        for prec in ("fp32", "fp16"):
            autotune.set_targets(case.op, 1, prec, 0, 0)


def test_batched_solve_with_tuned_totals_matches_oracle():
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import autotune
    ws = [synth.Workload(f"tb-{k}", 24, 0.222, 6, 1500, 2e-6, 4.0, 16, 100.0, 15.0, 6, "db4", 2, 700 + k,
                         z0=0.003 * k) for k in range(3)]
    cases = [Case(w, sh=True) for w in ws]
    ops = [solve.Operator(c.smaps, c.coef, c.time, c.basis_np, c.dw0, c.w.n) for c in cases]
    ys = [c64(o.A(c.x_noisy)) for o, c in zip(ops, cases)]
    try:
        # a large forward target and a small adjoint target: the group of 3 splits differently from 1
        autotune.set_targets(cases[0].op, 1, "fp32", 8192, 256)
        one = autotune.plan_info(cases[0].op, 1, "fp32", 1)
        three = autotune.plan_info(cases[0].op, 1, "fp32", 3)
        print(f"[case] tuned totals: P=1 {one}  P=3 {three}", flush=True)
        assert three["fwd_split"] <= one["fwd_split"]
        L = 1.05 * max(solve.power_lipschitz(o, c64(synth.power_start(w.npix, 3)), 20) for o, w in zip(ops, ws))
        xs = ee.fista_batched([c.to_dev(y) for c, y in zip(cases, ys)], [c.op for c in cases], 6, 2, "db4",
                              lipschitz=L, lam=1e-3)
        for k in range(3):
            ref = solve.fista(ops[k], ys[k], L, 1e-3, 6, 2, "db4", ws[k].n_pad)
            assert solve.nrmse(xs[k].cpu().numpy().reshape(-1), ref) <= 1e-5
    finally:
        autotune.set_targets(cases[0].op, 1, "fp32", 0, 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_column_width_one_keeps_parity(prec):
    """The tuner's other dimension: with 32 coils (two 16-column groups) a
    wave may carry one group instead of two (the groups then go to separate
    workgroups).  Under width 1 the plan reports it, A and A^H stay within
    the form's bar against the FP64 oracle, and an 8-iteration FISTA solve
    (operand builds, residual packing and the coil-combining reduction over
    two column groups) matches the oracle's."""
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import autotune
    w = synth.Workload("gw1", 32, 0.222, 32, 2000, 2e-6, 2.0, 16, 80.0, 20.0, 8, "db4", 2, 93, z0=0.001)
    case = Case(w, sh=True)
    try:
        assert autotune.plan_info(case.op, 1, prec)["col_groups"] == 2
        autotune.set_targets(case.op, 1, prec, 0, 0, 1)
        if prec != "fp32":
            autotune.set_targets(case.op, 1, "fp32", 0, 0, 1)
        info = autotune.plan_info(case.op, 1, prec)
        print(f"[case] width 1, {prec}: {info}", flush=True)
        assert info["col_groups"] == 1
        x = case.x_noisy
        y_ref = encoding.forward(x, *case.oracle_args())
        x_ref = encoding.adjoint(y_ref, *case.oracle_args())
        bar = 1e-5 if prec == "fp32" else 1e-3
        y = ee.forward(case.to_dev(x), case.op, prec).cpu().numpy()
        xa = ee.adjoint(case.to_dev(c64(y_ref)), case.op, prec).cpu().numpy()
        e_f, e_a = rel(y.reshape(y_ref.shape), y_ref), rel(xa.reshape(x_ref.shape), x_ref)
        print(f"  A {e_f:.2e}  A^H {e_a:.2e}", flush=True)
        assert e_f <= bar and e_a <= bar
        op = solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n)
        yd = c64(op.A(x))
        L = 1.05 * solve.power_lipschitz(op, c64(synth.power_start(w.npix, 4)), 30)
        r = ee.fista(case.to_dev(yd), case.op, 8, 2, "db4", precision=prec, lipschitz=L, lam=1e-3)
        ref = solve.fista(op, yd, L, 1e-3, 8, 2, "db4", w.n_pad)
        e = solve.nrmse(r.x.cpu().numpy().reshape(-1), ref)
        print(f"  FISTA 8 iterations: NRMSE vs oracle {e:.2e}", flush=True)
        assert e <= (1e-5 if prec == "fp32" else 1e-4)
    finally:
        autotune.set_targets(case.op, 1, prec, 0, 0, 0)
        autotune.set_targets(case.op, 1, "fp32", 0, 0, 0)
