"""Summaries of rocprofv3 output for the growth kernels.

Three commands, all reading CSV files that rocprofv3 wrote:

* ``stats``: turns ``*_kernel_stats.csv`` (from ``--kernel-trace --stats``)
  into a short markdown table (calls, total and average duration per
  kernel), headed by the command that produced it.
* ``traffic``: HBM bytes per launch of one kernel from two counter runs
  (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, both in KiB per
  dispatch), each scaled by what the same counter reads for a plain copy
  kernel of known size (``cg_test_copy``), stored in a JSON file keyed by
  workload and kernel label, together with a digest of the kernel sources so
  a reader can tell when the figure went stale.
* ``counters``: the same scaled FETCH/WRITE bytes for every kernel of a run,
  as a markdown table.
* ``sq``: SQ counters per kernel (VALU and LDS instructions, LDS active and
  bank-conflict cycles) with each kernel's average duration from a kernel
  trace of the same command, and its VALU fraction: wave-level VALU
  instructions over what 256 CUs issue at 2.4 GHz (one wave instruction per
  CU per cycle: four SIMD16 units, four cycles per wave64 instruction).

    python -m paper_2509_19162_amd.profiling stats --csv run_kernel_stats.csv \\
        --command "rocprofv3 ..." --out profiles/x.md
    python -m paper_2509_19162_amd.profiling traffic --workload pancake12 --label sort_pass \\
        --match onesweep_kernel --match ArraySrcT --fetch f.csv --write w.csv \\
        --copy-fetch cf.csv --copy-write cw.csv --copy-bytes 1073741824 --out profiles/traffic.json
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
from typing import Dict, List, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# device sources each measured kernel family is built from
KERNEL_SOURCES = {
    "sort_pass": ["radix_sort.hip", "device_util.h", "expand_device.h", "perm_rank.h"],
    "sort_pass_expand": ["radix_sort.hip", "device_util.h", "expand_device.h"],
    "dedup_compact": ["dedup.hip", "device_util.h", "perm_rank.h"],
    "expand": ["radix_sort.hip", "expand.hip", "expand_device.h", "perm_rank.h"],
    "digit_hist": ["radix_sort.hip", "expand_device.h"],
}


def source_digest(label: str) -> str:
    """sha256 prefix over the device sources of one kernel family."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(label, sorted(os.listdir(CSRC))):
        path = os.path.join(CSRC, name)
        if not os.path.exists(path):
            continue
        with open(path, "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(path: str) -> List[dict]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def counter_per_dispatch(path: str, counter: str, match: Sequence[str]) -> List[float]:
    """Counter values (summed over the rows of one dispatch) of every
    dispatch whose kernel name contains all of `match`."""
    per: Dict[str, float] = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        if not all(m in name for m in match):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per, key=lambda x: int(x))]


def cmd_stats(a) -> None:
    rows = _rows(a.csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# Kernel time: {a.title}", "", "Command:", "", "```", a.command, "```", ""]
    if a.note:
        out += [a.note, ""]
    out += ["| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows[: a.top]:
        name = r["Name"]
        short = name.replace("cg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        if len(short) > 90:
            short = short[:87] + "..."
        out.append(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")


def cmd_traffic(a) -> None:
    kib = 1024.0
    cf = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", ["copy_kernel"])
    cw = counter_per_dispatch(a.copy_write, "WRITE_SIZE", ["copy_kernel"])
    if not cf or not cw:
        sys.exit("no copy_kernel dispatches in the calibration runs")
    # the copy reads and writes copy_bytes each
    f_scale = a.copy_bytes / (sum(cf) / len(cf) * kib)
    w_scale = a.copy_bytes / (sum(cw) / len(cw) * kib)
    kf = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.match)
    kw = counter_per_dispatch(a.write, "WRITE_SIZE", a.match)
    if not kf or not kw:
        sys.exit("no matching dispatches in the kernel runs")
    fetch = sum(kf) / len(kf) * kib * f_scale
    write = sum(kw) / len(kw) * kib * w_scale
    entry = {
        "bytes_per_launch": round(fetch + write),
        "fetch_bytes_per_launch": round(fetch),
        "write_bytes_per_launch": round(write),
        "launches": len(kf),
        "copy_scale": {"fetch": round(f_scale, 4), "write": round(w_scale, 4),
                       "copy_bytes": a.copy_bytes},
        "match": list(a.match),
        "source_digest": source_digest(a.label),
        "commands": a.command or [],
    }
    d = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            d = json.load(f)
    d.setdefault(a.workload, {})[a.label] = entry
    with open(a.out, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(entry))


def cmd_counters(a) -> None:
    """Markdown table of scaled FETCH/WRITE bytes per kernel over a run."""
    kib = 1024.0
    f_scale = a.copy_bytes / (sum(counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", ["copy_kernel"])) /
                              len(counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", ["copy_kernel"])) * kib)
    w_scale = a.copy_bytes / (sum(counter_per_dispatch(a.copy_write, "WRITE_SIZE", ["copy_kernel"])) /
                              len(counter_per_dispatch(a.copy_write, "WRITE_SIZE", ["copy_kernel"])) * kib)
    tot: Dict[str, List[float]] = {}
    for path, counter, col, scale in ((a.fetch, "FETCH_SIZE", 1, f_scale), (a.write, "WRITE_SIZE", 2, w_scale)):
        seen = set()
        for r in _rows(path):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"].replace("cg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            e = tot.setdefault(name, [0.0, 0.0, 0.0])
            key = (name, r.get("Dispatch_Id"))
            if col == 1 and key not in seen:
                e[0] += 1
                seen.add(key)
            e[col] += float(r["Counter_Value"]) * kib * scale
    out = [f"# HBM traffic per kernel: {a.title}", "", "Commands:", "", "```"] + list(a.command or []) + ["```", "",
           f"Counter scale from the plain copy of {a.copy_bytes} bytes: FETCH_SIZE x {f_scale:.4f}, "
           f"WRITE_SIZE x {w_scale:.4f}.", ""]
    if a.note:
        out += [a.note, ""]
    out += ["| kernel | launches | fetch GB | write GB | GB per launch |", "|---|---:|---:|---:|---:|"]
    for name, (cnt, fb, wb) in sorted(tot.items(), key=lambda x: -(x[1][1] + x[1][2]))[: a.top]:
        per = (fb + wb) / cnt / 1e9 if cnt else 0.0
        out.append(f"| `{name[:90]}` | {int(cnt)} | {fb / 1e9:.3f} | {wb / 1e9:.3f} | {per:.4f} |")
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")


PEAK_WAVE_INSTR_PER_S = 256 * 2.4e9  # MI355X: one VALU wave instruction per CU per cycle


def cmd_sq(a) -> None:
    per: Dict[str, Dict[str, Dict[str, float]]] = {}
    for r in _rows(a.csv):
        name = r["Kernel_Name"].replace("cg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        d = per.setdefault(name, {}).setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    dur: Dict[str, List[float]] = {}
    for r in _rows(a.trace):
        name = r["Kernel_Name"].replace("cg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        dur.setdefault(name, []).append((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9)
    out = [f"# SQ counters per kernel: {a.title}", "", "Commands:", "", "```"] + list(a.command or []) + ["```", ""]
    if a.note:
        out += [a.note, ""]
    out += ["VALU fraction = SQ_INSTS_VALU / (average duration x 256 CUs x 2.4 GHz), durations from the kernel "
            "trace. LDS active = SQ_LDS_IDX_ACTIVE / (duration x 256 CUs x 2.4 GHz); conflict share = "
            "SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.", "",
            "| kernel | launches | VALU instr per launch | LDS instr per launch | avg ms | VALU fraction | "
            "LDS active | conflict share |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    rows = []
    for name, disp in per.items():
        n = len(disp)
        tot = {}
        for d in disp.values():
            for k, v in d.items():
                tot[k] = tot.get(k, 0.0) + v
        ds = dur.get(name)
        avg = sum(ds) / len(ds) if ds else 0.0
        valu = tot.get("SQ_INSTS_VALU", 0.0) / n
        lds = tot.get("SQ_INSTS_LDS", 0.0) / n
        act = tot.get("SQ_LDS_IDX_ACTIVE", 0.0) / n
        conf = tot.get("SQ_LDS_BANK_CONFLICT", 0.0) / n
        vf = valu / (avg * PEAK_WAVE_INSTR_PER_S) if avg else 0.0
        lf = act / (avg * PEAK_WAVE_INSTR_PER_S) if avg else 0.0
        rows.append((avg * len(ds or []), name, n, valu, lds, avg, vf, lf, conf / act if act else 0.0))
    for _, name, n, valu, lds, avg, vf, lf, cs in sorted(rows, reverse=True)[: a.top]:
        out.append(f"| `{name[:80]}` | {n} | {valu:.3e} | {lds:.3e} | {avg * 1e3:.3f} | {vf:.3f} | {lf:.3f} | {cs:.3f} |")
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(prog="python -m paper_2509_19162_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--note", default="")
    s.add_argument("--top", type=int, default=16)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--workload", required=True)
    t.add_argument("--label", required=True)
    t.add_argument("--match", action="append", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", action="append")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--title", default="")
    c.add_argument("--note", default="")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-fetch", required=True)
    c.add_argument("--copy-write", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--command", action="append")
    c.add_argument("--top", type=int, default=12)
    c.add_argument("--out", required=True)
    q = sub.add_parser("sq")
    q.add_argument("--title", default="")
    q.add_argument("--note", default="")
    q.add_argument("--csv", required=True, help="run_counter_collection.csv of the SQ counter run")
    q.add_argument("--trace", required=True, help="run_kernel_trace.csv of the same command")
    q.add_argument("--command", action="append")
    q.add_argument("--top", type=int, default=10)
    q.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters, "sq": cmd_sq}[a.cmd](a)


if __name__ == "__main__":
    main()
