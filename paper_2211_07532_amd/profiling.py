"""Profiling helpers (not part of the method): a small fixed workload to run
under ``rocprofv3 --pmc`` and summaries of rocprofv3's CSV output.

    # counters: one rocprofv3 pass per counter group, each on this workload
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -- \\
        python3 -m paper_2211_07532_amd.profiling run --forms fp32,fp16
    python3 -m paper_2211_07532_amd.profiling pmc OUT/*/*_counter_collection.csv

    # kernel durations grouped by kernel and launch grid
    python3 -m paper_2211_07532_amd.profiling trace OUT/*/*_kernel_trace.csv

    # effective shader clock per kernel: GRBM_GUI_ACTIVE (cycles, summed over
    # the 8 XCDs) over the dispatch's duration, from one run with both
    rocprofv3 --kernel-trace --pmc GRBM_GUI_ACTIVE GRBM_COUNT --output-format csv -d OUT -- \
        python3 -m paper_2211_07532_amd.profiling run --forms fp32,fp16 --repeat 10
    python3 -m paper_2211_07532_amd.profiling clock OUT/*/*_counter_collection.csv OUT/*/*_kernel_trace.csv

The workload copies a 256 MiB buffer (a plain copy of known size, the
calibration for byte counters) and applies A and A^H once per form to the
1.5 mm operator (148 x 148, 32 coils, 16384 samples, 16 field terms + dB0),
with the launch shapes of the autotuner's cache when it holds them.
"""
from __future__ import annotations

import argparse
import csv
import re
import sys
from collections import OrderedDict

COPY_BYTES = 256 << 20


def short_name(name: str) -> str:
    """'void expenc::k_adj_split_sh<2, false>(double const*, ...)' -> 'k_adj_split_sh<2, false>'."""
    n = re.sub(r"^void\s+", "", name.strip()).replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in n:
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        if ch == "(" and depth == 0:
            break
        out.append(ch)
    n = "".join(out)
    return n.split("::")[-1] if "expenc::" in n else n[:60]


def run(forms, repeat=1):
    import os
    import numpy as np
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth
    from . import expenc as ee
    from . import autotune
    w = synth.MM15
    dev = torch.device("cuda:0")
    p = synth.make_problem(w)

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    op = ee.Operator(w.n, w.n, t(p.smaps.astype(np.complex64)), t(p.coef), t(p.time), None, t(p.dw0),
                     sh_grid=(w.fov, w.fov, w.z0))
    x = t(p.x_noisy.astype(np.complex64))
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    for prec in forms:
        autotune.apply_cached(op, 1, prec)
        if prec != "fp32":
            autotune.apply_cached(op, 1, "fp32")
        for _ in range(repeat):
            y = ee.forward(x, op, prec)
            ee.adjoint(y, op, prec)
    torch.cuda.synchronize()
    print(f"profiling workload done: copy of {COPY_BYTES} bytes, A and A^H for {','.join(forms)}", flush=True)


def trace(paths):
    rows = OrderedDict()
    for path in paths:
        for r in csv.DictReader(open(path)):
            grid = (r.get("Grid_Size_X"), r.get("Grid_Size_Y"), r.get("Grid_Size_Z"))
            key = (short_name(r["Kernel_Name"]), "x".join(g for g in grid if g))
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            rows.setdefault(key, []).append(d)
    print("| kernel | grid (work-items) | calls | avg us | min us | max us |")
    print("|---|---|---|---|---|---|")
    for (k, g), v in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        print(f"| {k} | {g} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")


def pmc(paths):
    """Per (kernel, grid): mean of every counter over its dispatches.  Byte
    counters (FETCH_SIZE, WRITE_SIZE, in KiB) are also given scaled by the
    ratio of the copy's true bytes to its counter reading."""
    vals = OrderedDict()
    for path in paths:
        for r in csv.DictReader(open(path)):
            key = (short_name(r["Kernel_Name"]), r.get("Grid_Size", ""))
            vals.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    scale = {}
    for (k, g), cs in vals.items():
        if "copyBuffer" in k or "copy" in k.lower() and "k_copy" not in k:
            if "FETCH_SIZE" in cs:
                scale["FETCH_SIZE"] = COPY_BYTES / 1024 / max(cs["FETCH_SIZE"])
            if "WRITE_SIZE" in cs:
                scale["WRITE_SIZE"] = COPY_BYTES / 1024 / max(cs["WRITE_SIZE"])
    names = sorted({c for cs in vals.values() for c in cs})
    print("| kernel | grid | " + " | ".join(names) + " |")
    print("|---|---|" + "---|" * len(names))
    for (k, g), cs in vals.items():
        cells = []
        for n in names:
            if n not in cs:
                cells.append("")
                continue
            m = sum(cs[n]) / len(cs[n])
            cell = f"{m:.6g}"
            if n in scale:
                cell += f" ({m * scale[n] / 1024:.1f} MiB scaled)"
            cells.append(cell)
        print(f"| {k} | {g} | " + " | ".join(cells) + " |")
    if scale:
        print()
        print("copy calibration (true bytes / counter bytes): " +
              ", ".join(f"{k} x{v:.3f}" for k, v in scale.items()))


def clock(counter_csv, trace_csv, xcds=8):
    """Per (kernel, grid): GRBM_GUI_ACTIVE / xcds / duration, the shader clock
    the kernel ran at (MHz), averaged over its dispatches and over the later
    half of them (after the clock has settled)."""
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        dur[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    rows = OrderedDict()
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] != "GRBM_GUI_ACTIVE" or r["Dispatch_Id"] not in dur:
            continue
        key = (short_name(r["Kernel_Name"]), r.get("Grid_Size", ""))
        d = dur[r["Dispatch_Id"]]
        rows.setdefault(key, []).append((d, float(r["Counter_Value"]) / xcds / d / 1e6))
    print("| kernel | grid | dispatches | avg us | MHz (all) | MHz (later half) |")
    print("|---|---|---|---|---|---|")
    for (k, g), v in rows.items():
        late = v[len(v) // 2:]
        print(f"| {k} | {g} | {len(v)} | {1e6 * sum(d for d, _ in v) / len(v):.1f} | "
              f"{sum(m for _, m in v) / len(v):.0f} | {sum(m for _, m in late) / len(late):.0f} |")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2211_07532_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--forms", default="fp32,fp16")
    r.add_argument("--repeat", type=int, default=1)
    t = sub.add_parser("trace")
    t.add_argument("csv", nargs="+")
    c = sub.add_parser("pmc")
    c.add_argument("csv", nargs="+")
    k = sub.add_parser("clock")
    k.add_argument("counter_csv")
    k.add_argument("trace_csv")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run([f for f in a.forms.split(",") if f], a.repeat)
    elif a.cmd == "trace":
        trace(a.csv)
    elif a.cmd == "clock":
        clock(a.counter_csv, a.trace_csv)
    else:
        pmc(a.csv)


if __name__ == "__main__":
    main()
