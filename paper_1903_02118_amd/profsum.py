"""Summaries of rocprofv3 output for the committed `profiles/` folder.

    python -m paper_1903_02118_amd.profsum stats  <kernel_stats.csv> <out.md> --command "..."
    python -m paper_1903_02118_amd.profsum traffic <fetch_dir> <write_dir> <out.json> \
        --copy-bytes 1073741824 --last 100 --command-fetch "..." --command-write "..."

`stats` renders the per-kernel table of `rocprofv3 --kernel-trace --stats`.
`traffic` reads the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of two
`rocprofv3 --pmc` runs and calibrates each counter on a kernel of known
traffic in the same runs: FETCH_SIZE on the library's streaming-read probe
(`k_hbm_read`, which reads `--probe-bytes` once with the 16-byte
non-temporal loads of the near-field kernel), WRITE_SIZE on a plain
device-to-device copy of `--copy-bytes` (the probe writes nothing); then it
averages the last `--last` dispatches of each kernel (the steady state of the
run) and records the hash of the kernel sources so that a reader can drop
the figure once the kernels change.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# The per-step kernels whose counters a traffic summary records: a change to
# this source makes the stored counters stale.
HASHED = ("kernels.hip",)


def source_hash():
    h = hashlib.sha256()
    for f in HASHED:
        with open(os.path.join(ROOT, "paper_1903_02118_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    name = name.replace("(anonymous namespace)::", "")
    m = re.match(r"(?:void )?(?:bie::)?([A-Za-z_0-9]+(?:<[^()]*>)?)", name)
    return m.group(1) if m else name[:40]


def stats_md(csv_path, command, trace_path=None, tail=0):
    rows = list(csv.DictReader(open(csv_path)))
    tails = {}
    if trace_path and tail:
        per = {}
        for r in csv.DictReader(open(trace_path)):
            per.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        for k, v in per.items():
            if len(v) >= tail:
                tails[k] = sum(v[-tail:]) / tail
    hdr = "| kernel | calls | avg us | min us | max us | total % |"
    if tails:
        hdr += f" avg of last {tail} us |"
    out = [hdr, "|---" * (7 if tails else 6) + "|"]
    for r in rows:
        line = (
            f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
            f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | {float(r['Percentage']):.2f} |"
        )
        if tails:
            v = tails.get(r["Name"])
            line += f" {v/1e3:.1f} |" if v is not None else " |"
        out.append(line)
    return "\n".join(out)


def _dispatches(d):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(f[0])))


def traffic(fetch_dir, write_dir, copy_bytes, last, probe_bytes=None):
    res = {}
    cal = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _dispatches(d)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        probes = [float(r["Counter_Value"]) for r in rows if "k_hbm_read" in r["Kernel_Name"]]
        cal[key] = max(copies) if copies else None
        cal[key + "_probe"] = max(probes) if probes else None
        per = {}
        for r in rows:
            per.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        for k, v in per.items():
            tail = v[-last:]
            res.setdefault(k, {})[key + "_kib"] = sum(tail) / len(tail)
            res[k]["dispatches"] = len(v)
    out = {
        "source_hash": source_hash(),
        "copy_calibration": {
            "bytes_read": copy_bytes,
            "bytes_written": copy_bytes,
            "fetch_kib": cal["fetch"],
            "write_kib": cal["write"],
        },
        "averaged_over_last_dispatches": last,
        "kernels": {},
    }
    if probe_bytes and cal["fetch_probe"]:
        # reads calibrated on the probe: same loads as the kernels measured
        out["probe_calibration"] = {"bytes_read": probe_bytes, "fetch_kib": cal["fetch_probe"]}
        fs = probe_bytes / (cal["fetch_probe"] * 1024.0)
    else:
        fs = copy_bytes / (cal["fetch"] * 1024.0)
    ws = copy_bytes / (cal["write"] * 1024.0)
    for k, v in sorted(res.items(), key=lambda kv: kv[1]["dispatches"]):
        if "fetch_kib" in v and "write_kib" in v and k.startswith("k_"):
            # template variants of one kernel: keep the most dispatched one
            base = re.sub(r"<.*", "", k)
            out["kernels"][base] = {
                "dispatches": v["dispatches"],
                "name": k,
                "fetch_kib": v["fetch_kib"],
                "write_kib": v["write_kib"],
                "hbm_bytes": v["fetch_kib"] * 1024.0 * fs + v["write_kib"] * 1024.0 * ws,
            }
    out["scale_fetch"] = fs
    out["scale_write"] = ws
    return out


def traffic_md(t, title, alg_bytes=None, alg_kernel="k_near"):
    cal = t["copy_calibration"]
    pc = t.get("probe_calibration")
    if pc:
        caltext = (f"Calibration: the streaming-read probe `k_hbm_read` reads {pc['bytes_read']:,} bytes with the "
                   f"16-byte non-temporal loads of the near-field kernel and FETCH_SIZE counts {pc['fetch_kib']:.1f} "
                   f"KiB for it; a plain {cal['bytes_written']:,}-byte device-to-device copy counts WRITE_SIZE = "
                   f"{cal['write_kib']:.1f} KiB (FETCH_SIZE {cal['fetch_kib']:.1f} KiB).  FETCH_SIZE is scaled by "
                   f"{t['scale_fetch']:.4f} and WRITE_SIZE by {t['scale_write']:.4f}.")
    else:
        caltext = (f"Calibration: a plain {cal['bytes_read']:,}-byte device-to-device copy in the same runs reads "
                   f"FETCH_SIZE = {cal['fetch_kib']:.1f} KiB and WRITE_SIZE = {cal['write_kib']:.1f} KiB, so FETCH_SIZE "
                   f"is scaled by {t['scale_fetch']:.4f} and WRITE_SIZE by {t['scale_write']:.4f}.")
    out = [f"# {title}", "", "Commands (run from the repository root on one MI355X; one counter per run):", "", "```",
           t["command_fetch"], t["command_write"], "```", "", caltext,
           f"Values are averages over the last {t['averaged_over_last_dispatches']} dispatches of each kernel.", "",
           "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch |", "|---|---|---|---|"]
    for k, v in t["kernels"].items():
        out.append(f"| `{v['name']}` | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['hbm_bytes'] / 1e6:.1f} MB |")
    out.append("")
    k = t["kernels"].get(alg_kernel)
    if alg_bytes and k:
        out.append(f"Algorithmic bytes of `{alg_kernel}` per launch: {alg_bytes:,.0f} B; the counted traffic is "
                   f"{100.0 * (k['hbm_bytes'] / alg_bytes - 1.0):.1f}% above it.")
    out.append(f"Source hash of the kernels these counters belong to: `{t['source_hash']}` "
               "(bench.py reports `traffic` only while it matches).")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    a.add_argument("--trace", default=None, help="kernel_trace.csv of the same run (for the tail average)")
    a.add_argument("--tail", type=int, default=0, help="also report the average of the last N dispatches")
    a.add_argument("--note", default="")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--probe-bytes", type=int, default=None, help="bytes the k_hbm_read probe dispatch reads")
    b.add_argument("--last", type=int, default=100)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    b.add_argument("--md", default=None, help="also write a markdown summary here")
    b.add_argument("--title", default="HBM traffic per launch (rocprofv3 counters)")
    b.add_argument("--alg-bytes", type=float, default=None, help="algorithmic bytes per launch of --alg-kernel")
    b.add_argument("--alg-kernel", default="k_near")
    args = ap.parse_args()
    if args.cmd == "stats":
        body = stats_md(args.csv, args.command, args.trace, args.tail)
        with open(args.out, "w") as f:
            f.write(f"# {args.title}\n\nCommand (run from the repository root on one MI355X):\n\n```\n{args.command}\n```\n\n{body}\n")
            if args.note:
                f.write(f"\n{args.note}\n")
    else:
        t = traffic(args.fetch_dir, args.write_dir, args.copy_bytes, args.last, args.probe_bytes)
        t["command_fetch"] = args.command_fetch
        t["command_write"] = args.command_write
        with open(args.out, "w") as f:
            json.dump(t, f, indent=1)
            f.write("\n")
        if args.md:
            with open(args.md, "w") as f:
                f.write(traffic_md(t, args.title, args.alg_bytes, args.alg_kernel))


if __name__ == "__main__":
    main()
