"""Summarise rocprofv3 output into the text files under profiles/.

  python profile_summary.py trace  <kernel_stats.csv> <out.md> <command...>
  python profile_summary.py trace-variants <kernel_stats.csv> <out.md> <command...>
      (adds per-variant averages from the run_kernel_trace.csv beside it; for a
      run of the float64 forward step only, whose dispatch order is fixed)
  python profile_summary.py traffic <fetch counter_collection.csv> <write counter_collection.csv> <out.md> <command...>
  python profile_summary.py counters <csv,csv,...> <out.md> <kernel prefix,...> <command...>
      (per-dispatch averages of SQ counters from --pmc runs)
  (after the mode, --workload=periodic|channel|channel_cg picks the kernel-variant table and
  --cells=N records the cell count of the profiled field; bench.py uses a record only for that size)

`traffic` also updates profiles/traffic.json, the measured HBM bytes per
launch that bench.py reports as roofline.traffic (a list of records per
kernel variant, one per profiled field size). Counters are calibrated with
the library's plain copy kernel (k_stream_copy, bytes known): the measured
FETCH_SIZE and WRITE_SIZE of every kernel are scaled by
(bytes the copy moved) / (what the counter read for it). A record carries a
hash of the kernel's source files and is ignored once they change.

Per-variant records: one template instance can serve several launch variants
(the RK stage kernel runs as `stage` twice and `stage_last` once per step);
their dispatches interleave in a fixed order, given in VARIANT_ORDER.
"""
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2604_18536_amd", "csrc")

# template instance (prefix of the demangled name) -> (variant names in dispatch order, source files),
# per workload: the same kernel serves different steps on the periodic grid and on the channel
# (the strided FFT pass is y there, z here), so channel records carry a "channel:" prefix.
_WALL = ["k_walls.hip", "k_common.hpp", "ins_internal.hpp"]
VARIANT_ORDERS = {
    "periodic": {
        "void ins::k_stage_zm<double, true, 64, 8, double, false, 1>": (["stage_rec"], ["k_stage3d.hip", "k_common.hpp"]),
        "void ins::k_stage_zm<double, true, 64, 8, double, false, 2>": (["stage_last"], ["k_stage3d.hip", "k_common.hpp"]),
        "void ins::k_stage_zm<double, true, 64, 8, double, true, 3>": (["stage_yw"], ["k_stage3d.hip", "k_common.hpp"]),
        "void ins::k_stage_zm<double, false,": (["stage_first_rec"], ["k_stage3d.hip", "k_common.hpp"]),
        "void ins::k_fft_x_fwd<double, 3, 0,": (["fft_x_fwd_div"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_strided<0,": (["fft_y_fwd"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_strided<2,": (["fft_z_solve"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_strided<1,": (["fft_y_inv"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_x_inv<": (["fft_x_inv"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_apply_projection<double, 3,": (["apply_projection"], ["k_stencil.hip", "k_common.hpp"]),
    },
    # channel, direct pressure solve (FFTs along x and z, tridiagonal solves along y)
    "channel": {
        "void ins::k_wall_stage_zm<double, true,": (["channel:stage", "channel:stage", "channel:stage_last"], _WALL),
        "void ins::k_wall_stage_zm<double, false,": (["channel:stage_first"], _WALL),
        "void ins::k_fft_x_fwd<double, 3, 3,": (["channel:fft_x_fwd_div"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_strided<0,": (["channel:fft_z_fwd"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_channel_ysolve<": (["channel:channel_ysolve"], ["k_chsolve.hip", "k_common.hpp"]),
        "void ins::k_fft_strided<1,": (["channel:fft_z_inv"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_fft_x_inv<": (["channel:fft_x_inv"], ["k_fft.hip", "k_common.hpp"]),
        "void ins::k_wall_project<double, 3, false>": (["channel:wall_projection"], _WALL),
    },
    # channel, conjugate-gradient pressure solve: the two kernels of an iteration
    "channel_cg": {
        "ins::k_cg_apply3": (["channel:cg_apply"], _WALL),
        "void ins::k_cg_update<512, 3>": (["channel:cg_update"], _WALL),
    },
}
VARIANT_ORDER = VARIANT_ORDERS["periodic"]
COPY = "ins::k_stream_copy"


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace(stats_csv, out_md, command, variants=False, order=None):
    order = order or VARIANT_ORDER
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# rocprofv3 kernel trace summary", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if variants:
        # per launch variant (one template instance serves several, in a fixed dispatch order)
        tpath = os.path.join(os.path.dirname(stats_csv), os.path.basename(stats_csv).replace("kernel_stats", "kernel_trace"))
        per = defaultdict(list)
        disp = defaultdict(list)
        for r in csv.DictReader(open(tpath)):
            disp[r["Kernel_Name"].split("(")[0]].append(
                (int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for inst, (vnames, _) in order.items():
            names = [k for k in disp if k == inst or (inst.endswith((",", "<")) and k.startswith(inst))]
            durs = [d for _, d in sorted(x for k in names for x in disp[k])]
            for i, d in enumerate(durs):
                per[vnames[i % len(vnames)]].append(d)
        lines += ["", "Per launch variant (dispatches of one template instance assigned in their fixed order):", "",
                  "| variant | launches | avg us |", "|---|---|---|"]
        for v, ds in per.items():
            lines.append(f"| {v} | {len(ds)} | {sum(ds) / len(ds) / 1e3:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    d = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d[r["Kernel_Name"].split("(")[0]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"]) * 1024.0))
    for k in d:
        d[k].sort()
    return d


def traffic(fetch_csv, write_csv, out_md, command, copy_bytes=None, order=None, cells=None):
    order = order or VARIANT_ORDER
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")
    # copy calibration: the copy kernel reads and writes copy_bytes each
    cf = [v for _, v in f[COPY]][1:]  # first launch is a warm-up of the same size
    cw = [v for _, v in w[COPY]][1:]
    if copy_bytes is None:
        copy_bytes = 2 << 30
    kf = copy_bytes / (sum(cf) / len(cf))
    kw = copy_bytes / (sum(cw) / len(cw))
    lines = ["# HBM traffic per launch from rocprofv3 counters", "", "Commands (one counter per run):", "", "```",
             command, "```", "",
             f"Calibration with the plain copy kernel (reads and writes {copy_bytes / 2**20:.0f} MiB): "
             f"FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f}.", "",
             "| kernel variant | launches | fetched MiB | written MiB | total MiB |", "|---|---|---|---|---|"]
    rec = {}
    jpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(jpath):
        rec = json.load(open(jpath))
    for inst, (variants, srcs) in order.items():
        # a key is the demangled name or, for kernels templated on the FFT plan, its prefix
        names = [k for k in f if k == inst or (inst.endswith((",", "<")) and k.startswith(inst))]
        if not names:
            continue
        fv = [v for _, v in sorted(x for k in names for x in f[k])]
        wv = [v for _, v in sorted(x for k in names for x in w.get(k, []))]
        per = defaultdict(lambda: [0.0, 0.0, 0])
        for i in range(min(len(fv), len(wv))):
            name = variants[i % len(variants)]
            per[name][0] += fv[i] * kf
            per[name][1] += wv[i] * kw
            per[name][2] += 1
        for name, (a, b, n) in per.items():
            lines.append(f"| `{names[0].replace('void ', '')}` as {name} | {n} | {a / n / 2**20:.1f} | {b / n / 2**20:.1f} | "
                         f"{(a + b) / n / 2**20:.1f} |")
            new = {"bytes_per_launch": round((a + b) / n), "fetch": round(a / n), "write": round(b / n),
                   "sources": srcs, "source_hash": source_hash(srcs), "cells": cells}
            # one record per profiled field size: replace the one of the same size
            old = rec.get(name, [])
            old = old if isinstance(old, list) else [old]
            rec[name] = [r for r in old if r.get("cells") != cells] + [new]
    open(out_md, "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(jpath, "w"), indent=1, sort_keys=True)


def counters(csv_paths, out_md, command, prefixes):
    """Per-dispatch averages of every counter in one or more counter_collection.csv files,
    for the kernels whose demangled names start with one of `prefixes`."""
    acc = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"].split("(")[0]
            if not any(name.startswith(px) for px in prefixes):
                continue
            acc[name][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[(name, r["Counter_Name"])].add(int(r["Dispatch_Id"]))
    names = sorted({c for k in acc for c in acc[k]})
    lines = ["# rocprofv3 SQ counters per dispatch", "", "Commands (one counter set per run):", "", "```", command,
             "```", "", "| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
    for k in sorted(acc):
        row = []
        for c in names:
            n = len(disp[(k, c)])
            row.append(f"{acc[k][c] / n:.4g}" if n else "-")
        lines.append(f"| `{k.replace('void ', '')}` | " + " | ".join(row) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    args = sys.argv[1:]
    order = VARIANT_ORDERS["periodic"]
    cells = None
    while len(args) > 1 and args[1].startswith("--"):
        key, val = args.pop(1)[2:].split("=", 1)
        if key == "workload":
            order = VARIANT_ORDERS[val]
        elif key == "cells":
            cells = int(val)
    mode = args[0]
    if mode in ("trace", "trace-variants"):
        trace(args[1], args[2], " ".join(args[3:]), variants=mode == "trace-variants", order=order)
    elif mode == "traffic":
        traffic(args[1], args[2], args[3], " ".join(args[4:]), order=order, cells=cells)
    elif mode == "counters":
        # counters <csv,csv,...> <out.md> <kernel prefix,prefix,...> <command...>
        counters(args[1].split(","), args[2], " ".join(args[4:]), args[3].split(","))
    else:
        raise SystemExit(__doc__)
