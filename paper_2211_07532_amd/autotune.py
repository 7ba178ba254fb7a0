"""Autotuner for the launch shapes of the two contraction kernels.

Both contractions split their reduction (over pixels for A, over samples for
A^H) into chunks so that one launch has about `target` workgroups; more
chunks fill the 256 compute units better but cost partial-sum traffic and a
longer reduction.  The column width is the other tunable: a wave carries one
or two 16-column groups of the coil columns (two share each phase tile;
one needs half the accumulators and spreads the groups over workgroups).
For one operator geometry (grid, coils, samples, basis terms and kind),
batch and precision, ``tune`` times whole forward and adjoint applications
(torch events on the launch stream) over a ladder of targets for each width,
keeps the fastest target per direction within each width and the width with
the smallest forward + adjoint time (the width is shared by both directions:
the operand layouts follow it), registers the result with the library
(``expenc_set_launch_shape``) and stores it in a JSON cache keyed by the GPU
architecture and compute-unit count and the geometry, so later processes
apply it without timing again (``apply_cached``).  ``tuning_defaults.json``
beside this module ships the shapes measured for the benchmark geometries on
an MI355X (regenerate with ``python -m paper_2211_07532_amd.autotune --out
FILE``); a user cache entry takes precedence.  A batched solve of P problems
of one geometry uses the tuned totals across its P problems.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import os
from typing import Dict, Optional, Sequence

import torch

from . import _binding as _b
from . import expenc as _e

CANDIDATES = (512, 1024, 2048, 3072, 4096, 6144, 8192, 12288)


def cache_path() -> str:
    return os.environ.get("EXPENC_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2211_07532_amd", "tuning.json")


DEFAULTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_defaults.json")


def device_tag(device) -> str:
    """GPU architecture and compute-unit count, e.g. 'gfx950_cu256'."""
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}_cu{p.multi_processor_count}".replace(" ", "_")


def _key(op: _e.Operator, batch: int, precision) -> str:
    kind = "sh" if op._c.basis_kind == _b.BASIS_SH else "maps"
    return (f"{device_tag(op.device)}/nx{op.nx}_ny{op.ny}_c{op.ncoils}_t{op.nsamples}_l{op.nbasis}_{kind}"
            f"_b{batch}_p{_e._prec(precision)}")


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    d = _load(path)
    d[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def set_targets(op: _e.Operator, batch: int, precision, fwd_target: int, adj_target: int,
                col_groups: int = 0) -> None:
    """Registers the workgroup targets (0: default) and the column width
    (16-column groups per wave, 1 or 2; 0: default) for op's geometry."""
    _b.check(_b.lib().expenc_set_launch_shape(ctypes.byref(op._c), batch, _e._prec(precision), int(fwd_target),
                                              int(adj_target), int(col_groups)), "expenc_set_launch_shape")


def plan_info(op: _e.Operator, batch: int = 1, precision="fp32", nprob: int = 1) -> dict:
    out = (ctypes.c_int64 * 7)()
    _b.check(_b.lib().expenc_plan_info_ex(ctypes.byref(op._c), batch, _e._prec(precision), nprob, out, 7),
             "expenc_plan_info_ex")
    return {"fwd_split": out[0], "adj_split": out[1], "fwd_workgroups": out[2], "adj_workgroups": out[3],
            "fwd_split_max": out[4], "adj_split_max": out[5], "col_groups": out[6]}


@dataclasses.dataclass
class TuneResult:
    fwd_target: int
    adj_target: int
    fwd_ms: float
    adj_ms: float
    timings: Dict[tuple, tuple]    # (column groups, target) -> (forward ms, adjoint ms)
    cached: bool = False
    col_groups: int = 0            # 0: the library's default width
    width_ms: Dict[int, float] = dataclasses.field(default_factory=dict)  # width -> best forward + adjoint ms


def apply_cached(op: _e.Operator, batch: int = 1, precision="fp32", path: Optional[str] = None,
                 defaults: bool = True):
    """Registers a cached result for this geometry if there is one (the user
    cache first, then the shipped table of measured defaults); returns it
    (or None)."""
    key = _key(op, batch, precision)
    e = _load(path or cache_path()).get(key)
    if not e and defaults:
        e = _load(DEFAULTS).get(key)
    if not e:
        return None
    gw = int(e.get("col_groups", 0))
    set_targets(op, batch, precision, e["fwd_target"], e["adj_target"], gw)
    return TuneResult(e["fwd_target"], e["adj_target"], e["fwd_ms"], e["adj_ms"], {}, cached=True, col_groups=gw)


def _time_calls(fn, reps: int) -> float:
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()                    # plans, workspace and first-launch costs outside the timing
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps


def tune(op: _e.Operator, batch: int = 1, precision="fp32", candidates: Sequence[int] = CANDIDATES,
         reps: int = 5, path: Optional[str] = None, use_cache: bool = True, seed: int = 0,
         widths: Optional[Sequence[int]] = None) -> TuneResult:
    """Times forward and adjoint applications for each column width and
    workgroup target; registers the fastest target per direction of the
    width with the smallest forward + adjoint time.  Candidates that yield
    the same split as an earlier one of the same width are skipped.  widths
    defaults to (2, 1) when the coil columns span at least two 16-column
    groups, else the single width 1."""
    path = path or cache_path()
    if use_cache:
        r = apply_cached(op, batch, precision, path)
        if r is not None:
            return r
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((batch, op.npix, 2), generator=g).to(op.device)
    x = torch.view_as_complex(x.contiguous())
    if widths is None:
        widths = (2, 1) if batch * op.ncoils > 16 else (1,)
    timings: Dict[tuple, tuple] = {}
    width_ms: Dict[int, float] = {}
    best = None
    for gw in widths:
        set_targets(op, batch, precision, 0, 0, gw)
        y = _e.forward(x, op, precision)
        seen_f, seen_a = set(), set()
        for t in candidates:
            set_targets(op, batch, precision, t, t, gw)
            info = plan_info(op, batch, precision)
            tf = ta = float("inf")
            if info["fwd_split"] not in seen_f:
                seen_f.add(info["fwd_split"])
                tf = _time_calls(lambda: _e.forward(x, op, precision, out=y), reps)
            if info["adj_split"] not in seen_a:
                seen_a.add(info["adj_split"])
                ta = _time_calls(lambda: _e.adjoint(y, op, precision), reps)
            timings[(gw, t)] = (tf, ta)
        mine = [k for k in timings if k[0] == gw]
        bf = min(mine, key=lambda k: timings[k][0])
        ba = min(mine, key=lambda k: timings[k][1])
        total = timings[bf][0] + timings[ba][1]
        width_ms[gw] = total
        if best is None or total < best[0]:
            best = (total, gw, bf[1], ba[1], timings[bf][0], timings[ba][1])
    _, gw, best_f, best_a, fms, ams = best
    set_targets(op, batch, precision, best_f, best_a, gw)
    res = TuneResult(best_f, best_a, fms, ams, timings, col_groups=gw, width_ms=width_ms)
    _store(path, _key(op, batch, precision), {"fwd_target": best_f, "adj_target": best_a, "col_groups": gw,
                                              "fwd_ms": res.fwd_ms, "adj_ms": res.adj_ms})
    return res


def main(argv=None):
    """Times the launch shapes of the benchmark geometries on this GPU and
    writes them to a JSON file (the format of the shipped defaults)."""
    import argparse
    import sys
    import numpy as np
    ap = argparse.ArgumentParser(prog="python -m paper_2211_07532_amd.autotune")
    ap.add_argument("--out", required=True)
    ap.add_argument("--forms", default="fp32,bf16,fp16")
    ap.add_argument("--workloads", default="mm15,mm11,batch")
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    ws = []
    for name in a.workloads.split(","):
        if name == "mm15":
            ws.append(synth.MM15)
        elif name == "mm11":
            ws.append(synth.MM11)
        elif name == "batch":
            ws.extend(synth.batch_workloads(1, 3))
    dev = torch.device("cuda:0")
    for w in ws:
        p = synth.make_problem(w)

        def t(v):
            return torch.from_numpy(np.ascontiguousarray(v)).to(dev)

        op = _e.Operator(w.n, w.n, t(p.smaps.astype(np.complex64)), t(p.coef), t(p.time), None, t(p.dw0),
                         sh_grid=(w.fov, w.fov, w.z0))
        for f in a.forms.split(","):
            r = tune(op, 1, f, reps=10, path=a.out, use_cache=False)
            widths = ", ".join(f"{g}: {t:.4f}" for g, t in sorted(r.width_ms.items()))
            print(f"{w.name} {f}: column groups {r.col_groups}, forward target {r.fwd_target} "
                  f"({r.fwd_ms:.4f} ms), adjoint target {r.adj_target} ({r.adj_ms:.4f} ms); "
                  f"best A + A^H ms per width {{{widths}}}", flush=True)
            set_targets(op, 1, f, 0, 0)


if __name__ == "__main__":
    main()
