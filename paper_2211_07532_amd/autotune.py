"""Autotuner for the launch shapes of the two contraction kernels.

Both contractions split their reduction (over pixels for A, over samples for
A^H) into chunks so that one launch has about `target` workgroups; more
chunks fill the 256 compute units better but cost partial-sum traffic and a
longer reduction.  For one operator geometry (grid, coils, samples, basis
terms and kind), batch and precision, ``tune`` times whole forward and
adjoint applications (torch events on the launch stream) over a ladder of
targets, keeps the fastest per direction, registers it with the library
(``expenc_set_tuning``) and stores it in a JSON cache keyed by the device
name and the geometry, so later processes apply it without timing again
(``apply_cached``).  A batched solve of P problems of that geometry uses the
tuned totals across its P problems.
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


def _key(op: _e.Operator, batch: int, precision) -> str:
    name = torch.cuda.get_device_name(op.device).replace(" ", "_")
    kind = "sh" if op._c.basis_kind == _b.BASIS_SH else "maps"
    return (f"{name}/nx{op.nx}_ny{op.ny}_c{op.ncoils}_t{op.nsamples}_l{op.nbasis}_{kind}"
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


def set_targets(op: _e.Operator, batch: int, precision, fwd_target: int, adj_target: int) -> None:
    _b.check(_b.lib().expenc_set_tuning(ctypes.byref(op._c), batch, _e._prec(precision), int(fwd_target),
                                        int(adj_target)), "expenc_set_tuning")


def plan_info(op: _e.Operator, batch: int = 1, precision="fp32", nprob: int = 1) -> dict:
    out = (ctypes.c_int64 * 6)()
    _b.check(_b.lib().expenc_plan_info(ctypes.byref(op._c), batch, _e._prec(precision), nprob, out),
             "expenc_plan_info")
    return {"fwd_split": out[0], "adj_split": out[1], "fwd_workgroups": out[2], "adj_workgroups": out[3],
            "fwd_split_max": out[4], "adj_split_max": out[5]}


@dataclasses.dataclass
class TuneResult:
    fwd_target: int
    adj_target: int
    fwd_ms: float
    adj_ms: float
    timings: Dict[int, tuple]      # target -> (forward ms, adjoint ms)
    cached: bool = False


def apply_cached(op: _e.Operator, batch: int = 1, precision="fp32", path: Optional[str] = None):
    """Registers a cached result for this geometry if there is one; returns it (or None)."""
    e = _load(path or cache_path()).get(_key(op, batch, precision))
    if not e:
        return None
    set_targets(op, batch, precision, e["fwd_target"], e["adj_target"])
    return TuneResult(e["fwd_target"], e["adj_target"], e["fwd_ms"], e["adj_ms"], {}, cached=True)


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
         reps: int = 5, path: Optional[str] = None, use_cache: bool = True, seed: int = 0) -> TuneResult:
    """Times forward and adjoint applications for each workgroup target and
    registers the fastest per direction.  Candidates that yield the same
    split as an earlier one are skipped."""
    path = path or cache_path()
    if use_cache:
        r = apply_cached(op, batch, precision, path)
        if r is not None:
            return r
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((batch, op.npix, 2), generator=g).to(op.device)
    x = torch.view_as_complex(x.contiguous())
    y = _e.forward(x, op, precision)
    timings: Dict[int, tuple] = {}
    seen_f, seen_a = set(), set()
    for t in candidates:
        set_targets(op, batch, precision, t, t)
        info = plan_info(op, batch, precision)
        tf = ta = float("inf")
        if info["fwd_split"] not in seen_f:
            seen_f.add(info["fwd_split"])
            tf = _time_calls(lambda: _e.forward(x, op, precision, out=y), reps)
        if info["adj_split"] not in seen_a:
            seen_a.add(info["adj_split"])
            ta = _time_calls(lambda: _e.adjoint(y, op, precision), reps)
        timings[t] = (tf, ta)
    best_f = min(timings, key=lambda t: timings[t][0])
    best_a = min(timings, key=lambda t: timings[t][1])
    set_targets(op, batch, precision, best_f, best_a)
    res = TuneResult(best_f, best_a, timings[best_f][0], timings[best_a][1], timings)
    _store(path, _key(op, batch, precision), {"fwd_target": best_f, "adj_target": best_a,
                                              "fwd_ms": res.fwd_ms, "adj_ms": res.adj_ms})
    return res
