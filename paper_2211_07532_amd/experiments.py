"""Synthetic analogue of the paper's simulation study (Methods 2.2.2, Results,
Figs. 4 and 5): reconstructions of data simulated with the full expanded
encoding model, by least squares (CG with early stopping at 20 iterations)
and by CS (FISTA on eq. 1, 100 iterations), with

* the "expanded" model (all field terms and the B0 map),
* the "partial" model (no 2nd-order field terms),
* the model without the B0 map,

as a function of the acceleration factor, the number of virtual coils (32
physical coils compressed to 8 / 16 / 32) and the SNR (20 / 10 / 5), scored
by NRMSE against the noise-free object.  Everything runs on the GPU through
the library: data simulation (forward model), coil compression, power
iteration, lambda rule, CG and FISTA.

The object, coils and B0 map come from the seeded generators of the 1.5 mm
workload (148 x 148, FOV 222 mm, 32 coils, 1 us dwell, T = 3 N^2 / R so the
readout shortens with acceleration).  The field is the spiral k(t) in the
first-order terms plus smooth 0th/1st-order perturbations and 2nd-order
terms whose phase grows with the readout duration: their peak phase over
the FOV is `ho_frac` of the first-order phase range times T_read / 16.4 ms
(the R = 4 readout); no 3rd-order terms (the paper's field fit is 2nd order).

    python -m paper_2211_07532_amd.experiments fig4 --out fig4.json
    python -m paper_2211_07532_amd.experiments fig5 --out fig5.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time
from typing import Dict, List, Sequence

import numpy as np
import torch

from . import expenc as ee

N_2ND = 9          # basis terms up to 2nd order
T_REF = 16.4e-3    # s, the R = 4 readout of the 1.5 mm workload


def _synth():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    return synth


@dataclasses.dataclass
class Setting:
    accel: float
    vcoils: int
    snr: float


def workload(accel: float, snr: float, seed: int = 11, n: int = 148):
    """The simulation's workload: n x n (148 by default; smaller grids keep the
    FOV, so the pixels grow), T = 3 n^2 / R samples at 1 us."""
    synth = _synth()
    t = int(round(3 * n * n / accel))
    return synth.Workload(f"sim-R{accel:g}-snr{snr:g}", n, 0.222, 32, t, 1e-6, accel, N_2ND, 150.0, snr, 100,
                          "db4", 3, seed)


def field(w, ho_frac: float) -> np.ndarray:
    """coef [T][9]: the workload's spiral and 0th/1st-order perturbations;
    2nd-order terms rescaled to a peak phase of ho_frac * (first-order phase
    range) * T_read / T_REF."""
    synth = _synth()
    coef = synth.field_series(w)
    t_read = w.nsamples * w.dwell
    h = w.fov / 2
    rng_phase = np.pi * w.n / 2
    for l in range(4, N_2ND):
        peak = np.max(np.abs(coef[:, l])) * synth._SH_COEF_ABS[l] * h ** 2
        if peak > 0:
            coef[:, l] *= ho_frac * rng_phase * (t_read / T_REF) / peak
    return coef


def _t(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).cuda()


def simulate(accel: float, snr: float, ho_frac: float, seed: int = 11, n: int = 148):
    """(x_true [R], y [T][32], pieces) with y = A_exp x_noisy on the GPU."""
    synth = _synth()
    w = workload(accel, snr, seed, n)
    x_true = synth.phantom(w)
    x_noisy = x_true + synth.image_noise(w, x_true)
    smaps = synth.coil_maps(w)
    coef = field(w, ho_frac)
    tm = synth.sample_times(w)
    dw0 = synth.db0_map(w)
    op = ee.Operator(w.n, w.n, _t(smaps, np.complex64), _t(coef), _t(tm), None, _t(dw0),
                     sh_grid=(w.fov, w.fov, 0.0), nbasis=N_2ND)
    y = ee.forward(_t(x_noisy, np.complex64), op)
    return w, x_true, y, dict(smaps=op.smaps, coef=op.coef, time=op.time, dw0=op.dw0)


def operator(w, smaps, coef, tm, dw0, model: str):
    if model == "partial":
        coef = coef.clone()
        coef[:, 4:] = 0.0
    if model == "no_b0":
        dw0 = None
    return ee.Operator(w.n, w.n, smaps, coef, tm, None, dw0, sh_grid=(w.fov, w.fov, 0.0), nbasis=N_2ND)


def nrmse(x, ref) -> float:
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def reconstruct(w, y, op, method: str, precision: str, cs_iters: int, cg_iters: int):
    if method == "LS":
        return ee.cg(y, op, cg_iters, precision=precision)
    v0 = _t(_synth().power_start(w.npix, 7), np.complex64)
    return ee.fista(y, op, cs_iters, w.levels, w.wavelet, precision=precision, lipschitz=0.0, power_v0=v0,
                    n_power=20, lam=-1.0, lambda_factor=1e-3).x


def run(settings: Sequence[Setting], models=("expanded", "partial", "no_b0"), methods=("LS", "CS"),
        precision="fp32", cs_iters=100, cg_iters=20, ho_frac=0.005, seed=11) -> List[Dict]:
    out = []
    cache = {}
    for st in settings:
        key = (st.accel, st.snr)
        if key not in cache:
            cache = {key: simulate(st.accel, st.snr, ho_frac, seed)}
        w, x_true, y, p = cache[key]
        if st.vcoils < w.ncoils:
            yv, sv, _, _ = ee.coil_compress(y, st.vcoils, p["smaps"])
        else:
            yv, sv = y, p["smaps"]
        for model in models:
            op = operator(w, sv, p["coef"], p["time"], p["dw0"], model)
            for method in methods:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x = reconstruct(w, yv, op, method, precision, cs_iters, cg_iters)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                e = nrmse(x.cpu().numpy().reshape(-1).astype(np.complex128), x_true)
                out.append({"accel": st.accel, "vcoils": st.vcoils, "snr": st.snr, "model": model,
                            "method": method, "nrmse": e, "seconds": round(dt, 4)})
                print(f"R={st.accel:g} vc={st.vcoils} snr={st.snr:g} {model:9s} {method}: NRMSE {e:.4f} "
                      f"({dt * 1e3:.0f} ms)", flush=True)
    return out


def fig4(**kw):
    return run([Setting(a, 16, 20.0) for a in (2, 3, 4, 5, 6)], **kw)


def fig5(**kw):
    s = [Setting(a, vc, 20.0) for a in (2, 4, 6) for vc in (8, 16, 32)]
    s += [Setting(4, vc, snr) for snr in (10.0, 5.0) for vc in (8, 16, 32)]
    return run(s, models=("expanded",), **kw)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2211_07532_amd.experiments")
    ap.add_argument("which", choices=["fig4", "fig5"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--cs-iters", type=int, default=100)
    ap.add_argument("--ho-frac", type=float, default=0.005)
    a = ap.parse_args(argv)
    fn = fig4 if a.which == "fig4" else fig5
    res = fn(precision=a.precision, cs_iters=a.cs_iters, ho_frac=a.ho_frac)
    with open(a.out, "w") as f:
        json.dump({"experiment": a.which, "precision": a.precision, "ho_frac": a.ho_frac, "results": res}, f,
                  indent=1)


if __name__ == "__main__":
    main()
