"""Summaries of rocprofv3 output (CSV) for the measurement records.

    python -m paper_1907_11803_amd.profsum trace DIR --command CMD --title T --out FILE.md
    python -m paper_1907_11803_amd.profsum traffic --fetch DIR --write DIR --kernel NAME
        --calls N --workload TEXT --w W --probes P --probe-t T --sources F1,F2,..
        --command CMD --command CMD --out FILE.json
    python -m paper_1907_11803_amd.profsum counters DIR [DIR ...] --kernel NAME --command CMD
        --title T --out FILE.md

`trace` reads DIR/*kernel_trace.csv (rocprofv3 --kernel-trace --output-format
csv) and tabulates every kernel's dispatch count, duration and resources.
`traffic` reads the FETCH_SIZE and WRITE_SIZE passes (rocprofv3 --pmc ...
--output-format csv) of a profiling run of bench.py, which copies 1 GiB
device to device before its timed loop: that copy's counters give the scale
factors from counter units to bytes (a copy of 1 GiB reads and writes 1 GiB).
The named kernel's counters, summed over its dispatches and divided by the
number of query calls, give the HBM bytes of one step.  `counters` tabulates
any counters of one kernel, per grid size (so a build's large launches and a
query step's small ones stay apart).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 1 << 30


def source_hash(files) -> str:
    """Identifies a kernel's sources: a stored HBM traffic figure holds only
    while they are unchanged."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _csv(directory: str, suffix: str):
    paths = sorted(glob.glob(os.path.join(directory, f"*{suffix}")))
    if not paths:
        sys.exit(f"no *{suffix} under {directory}")
    rows = []
    for p in paths:
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _size(r, key: str) -> int:
    """Grid or workgroup size of a row (kernel traces split it into X/Y/Z)."""
    if key in r:
        return int(r[key])
    return int(r[key + "_X"]) * int(r.get(key + "_Y", 1) or 1) * int(r.get(key + "_Z", 1) or 1)


def _short(name: str, width: int = 90) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def cmd_trace(a):
    rows = _csv(a.dir, "kernel_trace.csv")
    by = collections.OrderedDict()
    for r in rows:
        by.setdefault(r["Kernel_Name"], []).append(r)
    out = [f"# {a.title}", "", "Command (from the repository root):", "", "```"]
    out += list(a.command) + ["```", "",
                              f"{len(rows)} dispatches in `{os.path.basename(a.dir)}/*kernel_trace.csv`.",
                              "", "| kernel | dispatches | mean us | min us | max us | total us | "
                              "workgroup | VGPR | AGPR | SGPR | LDS B | scratch B/lane |",
                              "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    items = []
    for name, rs in by.items():
        ds = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rs]
        items.append((sum(ds), name, rs, ds))
    for tot, name, rs, ds in sorted(items, key=lambda t: -t[0]):
        r = rs[0]
        out.append(f"| `{_short(name)}` | {len(ds)} | {statistics.mean(ds):.2f} | {min(ds):.2f} | "
                   f"{max(ds):.2f} | {tot:.1f} | {_size(r, 'Workgroup_Size')} | "
                   f"{r.get('VGPR_Count', '')} | {r.get('Accum_VGPR_Count', '')} | "
                   f"{r.get('SGPR_Count', '')} | {r.get('LDS_Block_Size', '')} | "
                   f"{r.get('Scratch_Size', '')} |")
    if a.kernel:
        sel = [t for t in items if a.kernel in t[1]]
        if sel:
            _, name, rs, ds = sel[0]
            grids = collections.Counter(_size(r, "Grid_Size") // max(1, _size(r, "Workgroup_Size")) for r in rs)
            out += ["", f"`{_short(name)}`: mean {statistics.mean(ds):.2f} us over {len(ds)} dispatches "
                    f"(median {statistics.median(ds):.2f}); workgroups per dispatch "
                    + ", ".join(f"{g} x{c}" for g, c in sorted(grids.items())) + "."]
    stats = sorted(glob.glob(os.path.join(a.dir, "*kernel_stats.csv")))
    if stats:
        with open(stats[0], newline="") as f:
            srows = list(csv.DictReader(f))
        out += ["", f"rocprofv3 --stats summary (`{os.path.basename(stats[0])}`, first {min(15, len(srows))} "
                "rows by total time):", "", "| kernel | calls | average us | min us | max us | % |",
                "|---|---|---|---|---|---|"]
        for r in srows[:15]:
            out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {r['Percentage']} |")
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print(f"wrote {a.out}")


def _counter(rows, counter, match):
    """Per-dispatch value of one counter for the kernels whose name contains
    `match` (summed over the counter's instances within the dispatch)."""
    per = collections.defaultdict(float)
    names = {}
    for r in rows:
        if r["Counter_Name"] != counter or match not in r["Kernel_Name"]:
            continue
        d = int(r["Dispatch_Id"])
        per[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return per, names


def cmd_traffic(a):
    res = {}
    for tag, directory, counter in (("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")):
        rows = _csv(directory, "counter_collection.csv")
        kern, names = _counter(rows, counter, a.kernel)
        copy, _ = _counter(rows, counter, a.copy_kernel)
        if not kern or not copy:
            sys.exit(f"{counter}: no dispatch of '{a.kernel}' or of the copy '{a.copy_kernel}'")
        # the copy's largest dispatches are the 1 GiB copies
        cvals = sorted(copy.values())[-3:]
        res[tag] = {"kib_per_step": sum(kern.values()) / a.calls, "dispatches": len(kern),
                    "copy_kib": statistics.mean(cvals),
                    "kernel": sorted(set(names.values()))}
    fetch_factor = COPY_BYTES / 1024 / res["fetch"]["copy_kib"]
    write_factor = COPY_BYTES / 1024 / res["write"]["copy_kib"]
    fb = res["fetch"]["kib_per_step"] * 1024 * fetch_factor
    wb = res["write"]["kib_per_step"] * 1024 * write_factor
    doc = {
        "kernel": a.kernel, "kernel_names": res["fetch"]["kernel"],
        "workload": a.workload, "w": a.w, "probes": a.probes,
        "probe_t": a.probe_t if a.probes == 2 else 0,
        "source": source_hash(a.sources.split(",")), "sources": a.sources.split(","),
        "calls": a.calls, "dispatches": res["fetch"]["dispatches"],
        "fetch_size_kib_per_step": round(res["fetch"]["kib_per_step"], 1),
        "write_size_kib_per_step": round(res["write"]["kib_per_step"], 1),
        "copy_1gib_fetch_size_kib": round(res["fetch"]["copy_kib"], 1),
        "copy_1gib_write_size_kib": round(res["write"]["copy_kib"], 1),
        "fetch_factor": round(fetch_factor, 4), "write_factor": round(write_factor, 4),
        "fetch_bytes_per_step": int(fb), "write_bytes_per_step": int(wb),
        "bytes_per_launch": int(fb + wb),
        "commands": list(a.command),
        "note": ("FETCH_SIZE and WRITE_SIZE in KiB per dispatch, summed over the kernel's dispatches "
                 "and divided by the query calls of the run (warm-up, timed and one statistics call; "
                 "every call runs the same step); scale factors from the 1 GiB device copy the "
                 "profiling run makes first."),
    }
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps(doc))


def cmd_counters(a):
    rows = []
    for d in a.dirs:
        rows.extend(_csv(d, "counter_collection.csv"))
    by_grid = collections.defaultdict(lambda: collections.defaultdict(list))
    names = set()
    per = collections.defaultdict(float)
    meta = {}
    for r in rows:
        if a.kernel not in r["Kernel_Name"]:
            continue
        key = (r["Dispatch_Id"], r["Counter_Name"], r.get("Start_Timestamp", ""))
        per[key] += float(r["Counter_Value"])
        meta[key] = (_size(r, "Grid_Size") // max(1, _size(r, "Workgroup_Size")), r["Kernel_Name"])
        names.add(r["Kernel_Name"])
    for key, v in per.items():
        grid, _ = meta[key]
        by_grid[grid][key[1]].append(v)
    out = [f"# {a.title}", "", "Commands (from the repository root):", "", "```"]
    out += list(a.command) + ["```", "", "Kernel: " + ", ".join(f"`{_short(n)}`" for n in sorted(names)), "",
                              "Mean per dispatch, by workgroups per dispatch:", ""]
    for grid in sorted(by_grid):
        cs = by_grid[grid]
        out += [f"## {grid} workgroups", "", "| counter | dispatches | mean per dispatch |", "|---|---|---|"]
        for c in sorted(cs):
            out.append(f"| {c} | {len(cs[c])} | {statistics.mean(cs[c]):.6g} |")
        out.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print(f"wrote {a.out}")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", required=True)
    t.add_argument("--kernel", default=None)
    t.add_argument("--out", required=True)
    t.set_defaults(fn=cmd_trace)
    p = sub.add_parser("traffic")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--copy-kernel", default="copy")
    p.add_argument("--calls", type=int, required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--w", type=float, required=True)
    p.add_argument("--probes", type=int, required=True)
    p.add_argument("--probe-t", type=int, default=0)
    p.add_argument("--sources", required=True)
    p.add_argument("--command", action="append", required=True)
    p.add_argument("--out", required=True)
    p.set_defaults(fn=cmd_traffic)
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--out", required=True)
    c.set_defaults(fn=cmd_counters)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == "__main__":
    main()
