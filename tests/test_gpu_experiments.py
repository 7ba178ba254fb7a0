"""The synthetic analogue of the paper's simulation study (Figs. 4 and 5)
reproduces the paper's qualitative findings on data simulated with the full
expanded model (148 px, 32 coils compressed to 16, SNR 20):

* the expanded model reconstructs better than the partial one (no 2nd-order
  terms), with a gap that shrinks as acceleration shortens the readout;
* CS with the expanded model has the lowest NRMSE at every acceleration;
* CS (100 FISTA iterations) costs several times the LS time (20 CG
  iterations), the paper's 5-10x.
The solvers themselves are parity-tested against the oracle elsewhere."""
import pytest

pytestmark = pytest.mark.gpu


def test_expanded_model_and_cs_win():
    from paper_2211_07532_amd import experiments as ex
    res = ex.run([ex.Setting(2, 16, 20.0), ex.Setting(4, 16, 20.0)], models=("expanded", "partial"))
    e = {(r["accel"], r["model"], r["method"]): r for r in res}
    for a in (2, 4):
        for m in ("LS", "CS"):
            assert e[(a, "expanded", m)]["nrmse"] < e[(a, "partial", m)]["nrmse"]
        best = min(r["nrmse"] for r in res if r["accel"] == a)
        assert e[(a, "expanded", "CS")]["nrmse"] == best
        assert e[(a, "expanded", "CS")]["seconds"] > 2.0 * e[(a, "expanded", "LS")]["seconds"]
    gap = {a: e[(a, "partial", "LS")]["nrmse"] - e[(a, "expanded", "LS")]["nrmse"] for a in (2, 4)}
    print(f"[case] partial - expanded (LS): R=2 {gap[2]:.4f}  R=4 {gap[4]:.4f}", flush=True)
    assert gap[2] > gap[4] > 0


def _oracle_inputs(accel, n, seed=11, ho_frac=0.005):
    """The simulation's inputs on the host (seeded generators, the same
    field recipe as the experiment) and the oracle's simulated data."""
    import numpy as np
    import synth
    from oracle import encoding
    from paper_2211_07532_amd import experiments as ex
    from tests.gpu_common import c64
    w = ex.workload(accel, 20.0, seed, n)
    x_true = synth.phantom(w)
    x_noisy = c64(x_true + synth.image_noise(w, x_true))
    smaps = c64(synth.coil_maps(w))
    coef = ex.field(w, ho_frac)
    tm = synth.sample_times(w)
    dw0 = synth.db0_map(w)
    basis = encoding.sh_basis(n, w.fov, 0.0, ex.N_2ND)
    y = encoding.forward(x_noisy, smaps, coef, tm, basis, dw0)
    return w, x_true, x_noisy, smaps, coef, tm, dw0, basis, np.ascontiguousarray(y)


def _gpu_operator(w, smaps, coef, tm, dw0, model):
    import numpy as np
    from paper_2211_07532_amd import experiments as ex
    return ex.operator(w, ex._t(smaps, np.complex64), ex._t(coef), ex._t(tm), ex._t(dw0), model)


def test_fig4_cell_matches_oracle_reduced_size():
    """One cell of the Fig. 4 analogue -- the partial model (no 2nd-order
    terms) at R = 4, LS by 20 CG iterations and CS by 100 FISTA iterations --
    on a 48 x 48 grid (T = 1728, 32 coils, no coil compression), through the
    experiment's own simulation and reconstruction calls, against the FP64
    oracle on the same inputs: the simulated data (expanded model) within
    1e-5, the CS image within 1e-5 and the cell's NRMSE within 1e-4 of the
    oracle's; 20-iteration CG (which amplifies rounding, see the CG tests)
    within 1e-2 and its NRMSE within 1e-3."""
    import numpy as np
    from oracle import solve
    from paper_2211_07532_amd import experiments as ex
    from tests.gpu_common import c64, rel
    import synth
    n = 48
    w, x_true, x_noisy, smaps, coef, tm, dw0, basis, y = _oracle_inputs(4, n)
    print(f"[case] Fig. 4 cell, partial model, R=4, {n}x{n}, T={w.nsamples}", flush=True)
    w_gpu, xt_gpu, y_gpu, _ = ex.simulate(4, 20.0, 0.005, 11, n)
    e_sim = rel(y_gpu.cpu().numpy(), y)
    coef_p = coef.copy()
    coef_p[:, 4:] = 0.0
    op = solve.Operator(smaps, coef_p, tm, basis, dw0, n)
    yc = c64(y)
    y_dev = ex._t(yc, np.complex64)
    gop = _gpu_operator(w, smaps, coef, tm, dw0, "partial")
    x_ls = ex.reconstruct(w, y_dev, gop, "LS", "fp32", 100, 20).cpu().numpy().reshape(-1)
    x_cs = ex.reconstruct(w, y_dev, gop, "CS", "fp32", 100, 20).cpu().numpy().reshape(-1)
    ref_ls = solve.cg_ls(op, yc, 20)
    L = solve.power_lipschitz(op, c64(synth.power_start(w.npix, 7)), 20)
    lam = solve.lambda_rule(op, yc)
    ref_cs = solve.fista(op, yc, L, lam, 100, w.levels, w.wavelet, w.n_pad)
    e_ls, e_cs = rel(x_ls, ref_ls), rel(x_cs, ref_cs)
    cell = {m: (ex.nrmse(x.astype(np.complex128), x_true), ex.nrmse(r, x_true))
            for m, x, r in (("LS", x_ls, ref_ls), ("CS", x_cs, ref_cs))}
    print(f"  simulated data {e_sim:.2e}; LS image {e_ls:.2e}, CS image {e_cs:.2e}; cell NRMSE (gpu, oracle): "
          f"{cell}", flush=True)
    assert e_sim <= 1e-5
    assert e_cs <= 1e-5 and abs(cell["CS"][0] - cell["CS"][1]) <= 1e-4
    assert e_ls <= 1e-2 and abs(cell["LS"][0] - cell["LS"][1]) <= 1e-3
    assert cell["CS"][1] < cell["LS"][1]   # the oracle's cell shows CS ahead of LS too


def test_cg_10_iterations_148px_matches_oracle():
    """LS at the experiment's full grid (148 x 148, R = 4, T = 16428, 32 coils,
    expanded model): 10 CG iterations against the oracle's CG on the same
    data, within 1e-4 (the CG tests' bar at 10 iterations)."""
    import numpy as np
    from oracle import solve
    from paper_2211_07532_amd import experiments as ex
    from tests.gpu_common import c64, rel
    w, x_true, x_noisy, smaps, coef, tm, dw0, basis, y = _oracle_inputs(4, 148)
    print(f"[case] CG 10 iterations at 148 px, T={w.nsamples}", flush=True)
    yc = c64(y)
    gop = _gpu_operator(w, smaps, coef, tm, dw0, "expanded")
    x = ex.reconstruct(w, ex._t(yc, np.complex64), gop, "LS", "fp32", 100, 10).cpu().numpy().reshape(-1)
    ref = solve.cg_ls(solve.Operator(smaps, coef, tm, basis, dw0, 148), yc, 10)
    e = rel(x, ref)
    print(f"  CG 10 at 148 px: {e:.2e} (NRMSE vs truth gpu {ex.nrmse(x.astype(np.complex128), x_true):.4f}, "
          f"oracle {ex.nrmse(ref, x_true):.4f})", flush=True)
    assert e <= 1e-4
