#!/usr/bin/env python
"""Summaries of rocprofv3 output for the profiles/ folder and bench.py.

    python profile_summary.py stats <kernel_stats.csv> [--top N]
        Markdown table of a --kernel-trace --stats run (calls, total and
        average duration per kernel).

    python profile_summary.py dispatches <kernel_trace.csv> --kernel NAME
        Markdown table of one kernel's dispatches of a --kernel-trace run,
        grouped by launch size (workgroups): count, median and fastest
        duration.

    python profile_summary.py counters <fetch.csv> <write.csv> --calib-mib M
        Markdown table of HBM bytes per launch for every kernel of two --pmc
        runs (FETCH_SIZE, then WRITE_SIZE), scaled as below.

    python profile_summary.py traffic <fetch.csv> <write.csv> --kernel NAME
            --workload TEXT --calib-mib M --algorithmic-bytes B --out FILE
        HBM bytes per launch of one kernel from two --pmc runs (FETCH_SIZE,
        then WRITE_SIZE; counter_collection.csv files).  Each counter is
        scaled by what it reads for the device-to-device copies of M MiB that
        bench.py --calib-copy-mib M appends (__amd_rocclr_copyBuffer dispatches
        of that size), so that the figure is in bytes moved.  Writes the JSON
        bench.py reports as roofline.traffic, stamped with the digest of the
        kernel sources so that a later change to them voids it.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    if "rocprim" in n:
        n = "rocprim (scan / radix sort)"
    return n


def stats(path: str, top: int) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total (us) | average (us) | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{short_name(r['Name'])}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def dispatches(path: str, kernel: str) -> str:
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if short_name(r["Kernel_Name"]) != kernel:
            continue
        wg = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        per[wg].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    if not per:
        raise SystemExit(f"kernel {kernel} not in the trace")
    out = ["| workgroups | dispatches | median (us) | fastest (us) |", "|---:|---:|---:|---:|"]
    for wg in sorted(per):
        v = sorted(per[wg])
        out.append(f"| {wg} | {len(v)} | {v[len(v) // 2]:.1f} | {v[0]:.1f} |")
    return "\n".join(out)


def load_counter(path: str):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[short_name(r["Kernel_Name"])].append((float(r["Counter_Value"]), int(r["Grid_Size"])))
    return per


def calib_scale(per, mib: int) -> float:
    """Bytes moved per counter unit (KiB) from the largest copy dispatches."""
    vals = [v for v, _ in per.get("__amd_rocclr_copyBuffer", [])]
    if not vals:
        raise SystemExit("no calibration copies in the counter file")
    big = sorted(vals)[-3:]
    avg = sum(big) / len(big)
    return mib * 1024.0 / avg


def counters_table(fetch: str, write: str, mib: int, top: int) -> str:
    f = load_counter(fetch)
    w = load_counter(write)
    fs, ws = calib_scale(f, mib), calib_scale(w, mib)
    rows = []
    for k, fv in f.items():
        if k == "__amd_rocclr_copyBuffer":
            continue
        wv = [v for v, _ in w.get(k, [])]
        fk = sum(v for v, _ in fv) / len(fv)
        wk = sum(wv) / len(wv) if wv else 0.0
        rows.append((k, len(fv), fk, wk, (fk * fs + wk * ws) * 1024.0 / 1e6))
    rows.sort(key=lambda r: -r[4] * r[1])
    out = [f"FETCH_SIZE scale {fs:.3f}, WRITE_SIZE scale {ws:.3f} (from the {mib} MiB copies)", "",
           "| kernel | launches | FETCH_SIZE KiB/launch (raw) | WRITE_SIZE KiB/launch | HBM MB/launch (scaled) |",
           "|---|---:|---:|---:|---:|"]
    for k, n, fk, wk, mb in rows[:top]:
        out.append(f"| `{k}` | {n} | {fk:.1f} | {wk:.1f} | {mb:.1f} |")
    return "\n".join(out)


def traffic(a) -> dict:
    f = load_counter(a.fetch)
    w = load_counter(a.write)
    k = a.kernel
    if k not in f or k not in w:
        raise SystemExit(f"kernel {k} not in the counter files (have: {sorted(f)[:12]})")
    fs = calib_scale(f, a.calib_mib)
    ws = calib_scale(w, a.calib_mib)
    fv = [v for v, _ in f[k]]
    wv = [v for v, _ in w[k]]
    fk = sum(fv) / len(fv)
    wk = sum(wv) / len(wv)
    bytes_per_launch = (fk * fs + wk * ws) * 1024.0
    sys.path.insert(0, ROOT)
    from bench import kernel_source_digest
    return {"kernel": k, "workload": a.workload, "launches": len(fv), "bytes_per_launch": round(bytes_per_launch),
            "fetch_kib_per_launch_raw": round(fk, 1), "write_kib_per_launch_raw": round(wk, 1),
            "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
            "algorithmic_bytes_per_launch": a.algorithmic_bytes,
            "kernel_source_digest": kernel_source_digest(),
            "note": (f"FETCH_SIZE x {fs:.3f} + WRITE_SIZE x {ws:.3f} KiB per dispatch (scales from {a.calib_mib} MiB "
                     "device copies in the same runs), averaged over the kernel's dispatches")}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=20)
    dp = sub.add_parser("dispatches")
    dp.add_argument("csv")
    dp.add_argument("--kernel", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("--calib-mib", type=int, required=True)
    c.add_argument("--top", type=int, default=16)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--kernel", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--calib-mib", type=int, required=True)
    t.add_argument("--algorithmic-bytes", type=float, default=None)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.csv, a.top))
        return 0
    if a.cmd == "dispatches":
        print(dispatches(a.csv, a.kernel))
        return 0
    if a.cmd == "counters":
        print(counters_table(a.fetch, a.write, a.calib_mib, a.top))
        return 0
    res = traffic(a)
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
