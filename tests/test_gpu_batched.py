"""GPU parity of the batched solve (fista_solve_batched): many independent
problems of mixed sizes, fields, coil maps and slice positions in one call.

* small mixed batches: every size class's first problem against the FP64
  oracle's FISTA (L from the oracle's power iteration on the same start
  vector, lambda by the same rule), every problem against the single-problem
  entry point on the same inputs (a consistency check of the grouping);
* full size: the 1.5 mm problem solved inside a batch (grouped with a second
  148 px problem, beside a 170 px group) against the stored FP64 oracle
  reconstruction.
Bars: NRMSE <= 1e-5 (FP32 form), <= 1e-4 (split forms), L and lambda 1e-5."""
import dataclasses
import os

import numpy as np
import pytest

import synth
from oracle import solve
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mm15_fista.npz")


def _ee():
    import paper_2211_07532_amd as ee
    return ee


def _mixed_workloads(n_per=2, n_iter=10, levels=2):
    # three size classes with T ~ 3 N^2 / R, per-problem seeds and slice positions
    sizes = ((20, 4.0), (24, 5.0), (28, 6.0))
    zs = (-0.003, 0.0, 0.003)
    out = []
    for k in range(3 * n_per):
        n, accel = sizes[k % 3]
        t = int(round(3 * n * n / accel))
        out.append(synth.Workload(f"mix-{k}", n, 0.222, 6, t, 2e-6, accel, 16, 100.0, 15.0, n_iter, "db4",
                                  levels, 500 + k, z0=zs[(k // 3) % 3]))
    return out


def _oracle_op(case):
    return solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, case.w.n)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_mixed_batch_matches_oracle_and_single_solves(prec):
    ee = _ee()
    ws = _mixed_workloads()
    cases = [Case(w, sh=True) for w in ws]
    ops = [_oracle_op(c) for c in cases]
    ys = [c64(o.A(c.x_noisy)) for o, c in zip(ops, cases)]
    rmax = max(w.npix for w in ws)
    v0 = c64(synth.power_start(rmax, 11))
    n_power = 25
    print(f"[case] batched {prec}: {len(ws)} problems, sizes {[w.n for w in ws]}", flush=True)
    xs = ee.fista_batched([c.to_dev(y) for c, y in zip(cases, ys)], [c.op for c in cases], ws[0].n_iter,
                          ws[0].levels, "db4", precision=prec, lipschitz=0.0, power_v0=cases[0].to_dev(v0),
                          n_power=n_power, lam=-1.0, lambda_factor=1e-3)
    bar = 1e-5 if prec == "fp32" else 1e-4
    for k in range(3):  # one oracle solve per size class
        w, op, y = ws[k], ops[k], ys[k]
        L = solve.power_lipschitz(op, v0[:w.npix], n_power)
        lam = solve.lambda_rule(op, y)
        ref = solve.fista(op, y, L, lam, w.n_iter, w.levels, w.wavelet, w.n_pad)
        e = solve.nrmse(xs[k].cpu().numpy().reshape(-1), ref)
        print(f"  problem {k} (n={w.n}): NRMSE vs oracle {e:.2e}", flush=True)
        assert e <= bar
    for k, (c, y) in enumerate(zip(cases, ys)):
        single = ee.fista(c.to_dev(y), c.op, ws[k].n_iter, ws[k].levels, "db4", precision=prec, lipschitz=0.0,
                          power_v0=c.to_dev(v0[:ws[k].npix]), n_power=n_power, lam=-1.0, lambda_factor=1e-3)
        e = rel(xs[k].cpu().numpy(), single.x.cpu().numpy())
        print(f"  problem {k}: batched vs single {e:.2e}", flush=True)
        assert e <= bar


@pytest.mark.parametrize("anchor", ["fp32", "ends"])
def test_batched_anchor_modes_match_oracle_and_single_solves(anchor):
    """The batched solver under the two other anchor modes (all anchors in
    FP32 at cadence 17; split anchors at cadence 5 with the last one in
    FP32), bf16: each size class against the FP64 oracle and every problem
    against its single solve with the same mode."""
    ee = _ee()
    ws = _mixed_workloads()
    cases = [Case(w, sh=True) for w in ws]
    ops = [_oracle_op(c) for c in cases]
    ys = [c64(o.A(c.x_noisy)) for o, c in zip(ops, cases)]
    rmax = max(w.npix for w in ws)
    v0 = c64(synth.power_start(rmax, 11))
    n_power = 25
    print(f"[case] batched bf16 anchor={anchor}: {len(ws)} problems", flush=True)
    xs = ee.fista_batched([c.to_dev(y) for c, y in zip(cases, ys)], [c.op for c in cases], ws[0].n_iter,
                          ws[0].levels, "db4", precision="bf16", lipschitz=0.0, power_v0=cases[0].to_dev(v0),
                          n_power=n_power, lam=-1.0, lambda_factor=1e-3, anchor=anchor)
    for k in range(3):
        w, op, y = ws[k], ops[k], ys[k]
        L = solve.power_lipschitz(op, v0[:w.npix], n_power)
        ref = solve.fista(op, y, L, solve.lambda_rule(op, y), w.n_iter, w.levels, w.wavelet, w.n_pad)
        e = solve.nrmse(xs[k].cpu().numpy().reshape(-1), ref)
        print(f"  problem {k} (n={w.n}): NRMSE vs oracle {e:.2e}", flush=True)
        assert e <= 1e-4
    for k, (c, y) in enumerate(zip(cases, ys)):
        single = ee.fista(c.to_dev(y), c.op, ws[k].n_iter, ws[k].levels, "db4", precision="bf16", lipschitz=0.0,
                          power_v0=c.to_dev(v0[:ws[k].npix]), n_power=n_power, lam=-1.0, lambda_factor=1e-3,
                          anchor=anchor)
        e = rel(xs[k].cpu().numpy(), single.x.cpu().numpy())
        print(f"  problem {k}: batched vs single {e:.2e}", flush=True)
        assert e <= 1e-4


def test_batched_fp16_scales_per_problem():
    """The fp16 form's operand scales are per problem: the problems of one
    launch (two per size class here) get data scaled by very different powers
    of two, and each solution must be its unscaled single solve times that
    factor (the scaling is exact, so to within rounding)."""
    ee = _ee()
    ws = _mixed_workloads(n_per=2, n_iter=8)
    cases = [Case(w, sh=True) for w in ws]
    ops = [_oracle_op(c) for c in cases]
    ys = [c64(o.A(c.x_noisy)) for o, c in zip(ops, cases)]
    factors = [2.0 ** e for e in (-20, 10, 0, -5, 15, -10)]
    v0 = c64(synth.power_start(max(w.npix for w in ws), 13))
    kw = dict(precision="fp16", lipschitz=0.0, power_v0=cases[0].to_dev(v0), n_power=20, lam=-1.0,
              lambda_factor=1e-3)
    xs = ee.fista_batched([c.to_dev(y * f) for c, y, f in zip(cases, ys, factors)], [c.op for c in cases],
                          ws[0].n_iter, ws[0].levels, "db4", **kw)
    for k, (c, y, f) in enumerate(zip(cases, ys, factors)):
        single = ee.fista(c.to_dev(y), c.op, ws[k].n_iter, ws[k].levels, "db4",
                          **dict(kw, power_v0=c.to_dev(v0[:ws[k].npix])))
        e = rel(xs[k].cpu().numpy() / f, single.x.cpu().numpy())
        print(f"  problem {k} (n={ws[k].n}, data x{f:g}): batched / factor vs single unscaled {e:.2e}", flush=True)
        assert e <= 1e-6


def test_batched_fixed_scalars_and_repeat_is_bitwise():
    ee = _ee()
    ws = _mixed_workloads(n_per=1, n_iter=6)
    cases = [Case(w, sh=False) for w in ws]
    ops = [_oracle_op(c) for c in cases]
    ys = [c64(o.A(c.x_noisy)) for o, c in zip(ops, cases)]
    # one L that bounds every problem's Lipschitz constant, one fixed lambda
    L = 1.05 * max(solve.power_lipschitz(o, c64(synth.power_start(w.npix, 12)), 20) for o, w in zip(ops, ws))
    lam = 2e-3
    args = ([c.to_dev(y) for c, y in zip(cases, ys)], [c.op for c in cases], 6, 2, "db4")
    xs = ee.fista_batched(*args, lipschitz=L, lam=lam)
    for k in range(3):
        ref = solve.fista(ops[k], ys[k], L, lam, 6, 2, "db4", ws[k].n_pad)
        assert solve.nrmse(xs[k].cpu().numpy().reshape(-1), ref) <= 1e-5
    # the second call replays the cached graph
    xs2 = ee.fista_batched(*args, lipschitz=L, lam=lam)
    for a, b in zip(xs, xs2):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_concurrent_host_threads_match_calls_made_alone():
    """Four host threads issue batched solves at the same moment, each on its
    own stream with its own workspace (so each captures a graph of its own):
    the library's shared state (graph cache, capture stream, fork streams)
    must keep them apart, so that every result, first call and cached replay,
    is bitwise the same call made alone."""
    import ctypes
    import threading
    import torch
    from paper_2211_07532_amd import _binding as b
    ws_ = _mixed_workloads(n_per=1, n_iter=6)
    cases = [Case(w, sh=True) for w in ws_]
    ops = [_oracle_op(c) for c in cases]
    ys = [c.to_dev(c64(o.A(c.x_noisy))) for o, c in zip(ops, cases)]
    L = 1.05 * max(solve.power_lipschitz(o, c64(synth.power_start(w.npix, 12)), 20) for o, w in zip(ops, ws_))
    n = len(cases)
    carr = (b.ExpencOp * n)(*[c.op._c for c in cases])
    yp = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    precs = [b.FP16_SPLIT, b.FP32, b.FP16_SPLIT, b.BF16_SPLIT]

    def solve_once(prec, stream, ws, xs):
        opts = b.FistaOpts(6, prec, b.DB4, 2, 0, 0, 0, 0, 0, b.EXPENC_BATCH_FORKED, L, 2e-3, 0.0, None, None,
                           None)
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        return b.lib().fista_solve_batched(n, carr, 1, yp, xp, ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()),
                                           ws.numel(), ctypes.c_void_p(stream.cuda_stream))

    def resources(prec):
        opts = b.FistaOpts(6, prec, b.DB4, 2, 0, 0, 0, 0, 0, 0, L, 2e-3, 0.0, None, None, None)
        need = b.lib().fista_batched_workspace_size(n, carr, 1, ctypes.byref(opts))
        assert need > 0
        ws = torch.zeros(need, dtype=torch.uint8, device="cuda")
        runs = [[torch.zeros((c.w.n, c.w.n), dtype=torch.complex64, device="cuda") for c in cases] for _ in range(2)]
        return torch.cuda.Stream(), ws, runs

    res = [resources(p) for p in precs]
    torch.cuda.synchronize()
    rcs = [[None, None] for _ in precs]
    gate = threading.Barrier(len(precs))

    def worker(i):
        stream, ws, runs = res[i]
        gate.wait()
        for r in range(2):  # the first call captures, the second replays
            rcs[i][r] = solve_once(precs[i], stream, ws, runs[r])
        stream.synchronize()

    print(f"[case] {len(precs)} threads, batched solves of {n} problems each", flush=True)
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(precs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
        assert not t.is_alive()
    torch.cuda.synchronize()
    assert rcs == [[b.EXPENC_OK, b.EXPENC_OK]] * len(precs), rcs
    for i, p in enumerate(precs):
        stream, _, _ = res[i]
        ws = torch.zeros_like(res[i][1])
        alone = [torch.zeros_like(x) for x in res[i][2][0]]
        assert solve_once(p, stream, ws, alone) == b.EXPENC_OK
        stream.synchronize()
        for r in range(2):
            for a, x in zip(alone, res[i][2][r]):
                assert torch.equal(a.view(torch.float32), x.view(torch.float32)), (i, r)


def test_binding_threads_on_own_streams_share_an_operator():
    """Through the Python binding: threads that solve with ONE operator, each
    on its own torch stream, get workspaces of their own (the binding keys
    them by stream) and the result of the call made alone."""
    import threading
    import torch
    ee = _ee()
    w = _mixed_workloads(n_per=1, n_iter=6)[1]
    c = Case(w, sh=True)
    y0 = c64(_oracle_op(c).A(c.x_noisy))
    L = 1.05 * solve.power_lipschitz(_oracle_op(c), c64(synth.power_start(w.npix, 12)), 20)
    precs = ["fp16", "fp32", "fp16"]
    ys = [c.to_dev(y0 * (k + 1)) for k in range(len(precs))]
    kw = dict(lipschitz=L, lam=2e-3)
    streams = [torch.cuda.Stream() for _ in precs]
    out = [None] * len(precs)
    gate = threading.Barrier(len(precs))
    torch.cuda.synchronize()

    def worker(i):
        with torch.cuda.stream(streams[i]):
            gate.wait()
            out[i] = [ee.fista(ys[i], c.op, 6, 2, "db4", precision=precs[i], **kw).x for _ in range(2)]
        streams[i].synchronize()

    print(f"[case] {len(precs)} threads on one operator (n={w.n})", flush=True)
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(precs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
        assert not t.is_alive()
    torch.cuda.synchronize()
    for i, p in enumerate(precs):
        alone = ee.fista(ys[i], c.op, 6, 2, "db4", precision=p, **kw).x
        for r in range(2):
            assert torch.equal(alone.view(torch.float32), out[i][r].view(torch.float32)), (i, r)


def test_batched_rejects_bad_arguments():
    import ctypes
    import torch
    from paper_2211_07532_amd import _binding as b
    ee = _ee()
    w = _mixed_workloads(n_per=1)[0]
    c = Case(w, sh=True)
    y = torch.zeros((w.nsamples, 6), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ee.fista_batched([y], [c.op], 2, 2, lipschitz=0.0)      # no power start vector
    opts = b.FistaOpts(2, 0, 1, 2, 24, 24, 0, 0, 0, 0, 1.0, 1.0, 0.0, None, None, None)
    arr = (b.ExpencOp * 1)(c.op._c)
    assert b.lib().fista_batched_workspace_size(1, arr, 1, ctypes.byref(opts)) == 0  # padding is per problem
    opts.nx_pad = opts.ny_pad = 0
    assert b.lib().fista_batched_workspace_size(1, arr, 1, ctypes.byref(opts)) > 0
    yp = (ctypes.c_void_p * 1)(y.data_ptr())
    xp = (ctypes.c_void_p * 1)(None)
    st = b.lib().fista_solve_batched(1, arr, 1, yp, xp, ctypes.byref(opts), None, 0, None)
    assert st == b.EXPENC_EINVAL


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_full_size_problem_inside_batch_matches_golden(prec):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    import torch
    ee = _ee()
    g = np.load(GOLDEN)
    w = synth.MM15
    main = Case(w, sh=True)
    y = c64(solve.Operator(main.smaps, main.coef, main.time, main.basis_np, main.dw0, w.n).A(main.x_noisy))
    # batch partners: a second 148 px problem (same group) and a 170 px one
    bw = synth.batch_workloads(n_slices=1, n_vol=3)
    partners = [Case(dataclasses.replace(bw[0], n_iter=w.n_iter), sh=True),
                Case(dataclasses.replace(bw[1], n_iter=w.n_iter), sh=True)]
    yps = [ee.forward(p.to_dev(p.x_noisy), p.op) for p in partners]
    v0 = c64(synth.power_start(max(p.w.npix for p in partners + [main]), int(g["power_seed"])))
    v0[:w.npix] = c64(synth.power_start(w.npix, int(g["power_seed"])))
    print(f"[case] full-size batch {prec}: 148 (golden) + 148 + 170", flush=True)
    xs = ee.fista_batched([main.to_dev(y)] + yps, [main.op] + [p.op for p in partners], w.n_iter, w.levels,
                          w.wavelet, precision=prec, lipschitz=0.0, power_v0=main.to_dev(v0),
                          n_power=int(g["n_power"]), lam=-1.0, lambda_factor=1e-3)
    torch.cuda.synchronize()
    e = solve.nrmse(xs[0].cpu().numpy().reshape(-1), g["x_hat"])
    print(f"  golden NRMSE {e:.2e}", flush=True)
    assert e <= 1e-5
    for p, yp, x in zip(partners, yps, xs[1:]):
        single = ee.fista(yp, p.op, w.n_iter, w.levels, w.wavelet, precision=prec, lipschitz=0.0,
                          power_v0=main.to_dev(v0[:p.w.npix]), n_power=int(g["n_power"]), lam=-1.0,
                          lambda_factor=1e-3)
        e2 = rel(x.cpu().numpy(), single.x.cpu().numpy())
        print(f"  partner n={p.w.n}: batched vs single {e2:.2e}", flush=True)
        assert e2 <= (1e-5 if prec == "fp32" else 1e-4)


def test_full_size_twelve_per_launch_keeps_single_accuracy():
    """Twelve copies of the 1.5 mm golden problem in one group (one launch of
    each kernel for all twelve): the workgroup totals tuned for one problem
    would leave each copy a few long reduction chunks, and long sums on the
    matrix cores cost the split form accuracy (unbounded, the FP32 anchors'
    and the split adjoint's chunks took a 200 px solve from 1.9e-5 to
    6.1e-5); with the chunk caps every copy stays near the single solve."""
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    ee = _ee()
    g = np.load(GOLDEN)
    w = synth.MM15
    main = Case(w, sh=True)
    y = main.to_dev(c64(solve.Operator(main.smaps, main.coef, main.time, main.basis_np, main.dw0, w.n)
                        .A(main.x_noisy)))
    kw = dict(precision="fp16", lipschitz=float(g["lipschitz"]), lam=float(g["lam"]))
    xs = ee.fista_batched([y] * 12, [main.op] * 12, w.n_iter, w.levels, w.wavelet, **kw)
    single = ee.fista(y, main.op, w.n_iter, w.levels, w.wavelet, **kw).x
    e_single = solve.nrmse(single.cpu().numpy().reshape(-1), g["x_hat"])
    e = max(solve.nrmse(x.cpu().numpy().reshape(-1), g["x_hat"]) for x in xs)
    print(f"  12 per launch: worst NRMSE {e:.2e} (single {e_single:.2e})", flush=True)
    assert e <= max(2.0 * e_single, 2e-5)


def _many_groups(n_groups, n_iter, levels=2):
    # one problem per size class, so every problem is a group of its own
    out = []
    for k in range(n_groups):
        n = 16 + 4 * k
        t = int(round(3 * n * n / 4.0))
        out.append(synth.Workload(f"grp-{k}", n, 0.222, 6, t, 2e-6, 4.0, 16, 100.0, 15.0, n_iter, "db4",
                                  levels, 700 + k, z0=0.002 * (k % 3 - 1)))
    return out


@pytest.mark.parametrize("prec,n_groups", [("fp16", 3), ("bf16", 3), ("fp16", 10)])
def test_grouped_launch_is_bitwise_equal_to_forked(prec, n_groups):
    """The grouped contractions (every group's tiles in one launch
    per pass, groups in lock step) against each group's own launches on
    forked streams: the same tiles with the same arithmetic, so the results
    are bit-identical.  30 iterations cover the first gradient from the
    lambda rule, split-difference iterations, split anchors and the last
    iteration's FP32 anchor; 10 groups take
    two grouped launches per pass (at most 8 groups each)."""
    ee = _ee()
    ws = _many_groups(n_groups, 30) if n_groups > 3 else _mixed_workloads(n_per=2, n_iter=30)
    cases = [Case(w, sh=True) for w in ws]
    ys = [c.to_dev(c64(_oracle_op(c).A(c.x_noisy))) for c in cases]
    v0 = cases[0].to_dev(c64(synth.power_start(max(w.npix for w in ws), 17)))
    kw = dict(precision=prec, lipschitz=0.0, power_v0=v0, n_power=20, lam=-1.0, lambda_factor=1e-3,
              check_status=True)
    print(f"[case] grouped vs forked {prec}: {len(ws)} problems, sizes {sorted({w.n for w in ws})}", flush=True)
    xf = ee.fista_batched(ys, [c.op for c in cases], 30, 2, "db4", launch="forked", **kw)
    xg = ee.fista_batched(ys, [c.op for c in cases], 30, 2, "db4", launch="grouped", **kw)
    for k, (a, b) in enumerate(zip(xf, xg)):
        same = np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))
        if not same:
            print(f"  problem {k}: grouped vs forked {rel(b.cpu().numpy(), a.cpu().numpy()):.2e}", flush=True)
        assert same
    # the replayed graph of the grouped form gives the same result again
    xg2 = ee.fista_batched(ys, [c.op for c in cases], 30, 2, "db4", launch="grouped", **kw)
    for a, b in zip(xg, xg2):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_grouped_launch_rejects_unsupported_forms():
    from paper_2211_07532_amd import _binding as b
    ee = _ee()
    ws = _mixed_workloads(n_per=1, n_iter=4)
    for prec, sh in (("fp32", True), ("fp16", False)):
        cases = [Case(w, sh=sh) for w in ws]
        ys = [c.to_dev(c64(_oracle_op(c).A(c.x_noisy))) for c in cases]
        with pytest.raises(b.ExpencError) as ei:
            ee.fista_batched(ys, [c.op for c in cases], 4, 2, "db4", precision=prec, lipschitz=1e4, lam=1e-3,
                             launch="grouped")
        assert ei.value.status == b.EXPENC_EUNSUPPORTED
    with pytest.raises(ValueError):
        ee.fista_batched(ys, [c.op for c in cases], 4, 2, "db4", lipschitz=1e4, lam=1e-3, launch="queued")
