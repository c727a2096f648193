"""Condense rocprofv3 output into the short summaries kept under profiles/.

    # kernel durations (rocprofv3 --kernel-trace --stats ... --output-format csv)
    python -m paper_1803_00005_amd.profile_summary stats DIR OUT.md --command "..."

    # HBM bytes per launch from two counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE)
    python -m paper_1803_00005_amd.profile_summary counters FETCH_DIR WRITE_DIR OUT.json \
        --workload NAME --command "..."

The counter runs must include a known-size calibration (``bench.py
--copy-calibration``: a fill that writes 1 GiB and sums that read 1 GiB).
The calibration factors scale the raw counters to bytes: factor = known
bytes / counter bytes of the calibration kernel.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re

from .build_lib import source_hash

CAL_BYTES = 1 << 30
OURS = re.compile(r"hgf::")


def short_name(k: str) -> str:
    """'void hgf::coef_kernel<9, 1, 9, 0, float, 64>(...)' -> 'coef_kernel<9, 1, 9, 0, float, 64>'."""
    k = k.strip().replace("(anonymous namespace)::", "")
    if k.startswith("void "):
        k = k[5:]
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            k = k[:i]
            break
    return k.split("hgf::")[-1] if "hgf::" in k else k[:60]


def _find(d: str, suffix: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def stats(d: str, out: str, command: str) -> None:
    files = _find(d, "kernel_stats.csv")
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    lines = [
        "# Kernel durations",
        "",
        "Command (from the repository root on the GPU machine):",
        "",
        "```",
        command,
        "```",
        "",
        "| kernel | calls | average (us) | min (us) | max (us) | total (ms) | share |",
        "|---|---:|---:|---:|---:|---:|---:|",
    ]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['Percentage']):.1f}% |")
    lines += ["", f"Kernel sources: `{source_hash()}`", ""]
    with open(out, "w") as fh:
        fh.write("\n".join(lines))


def _counter(d: str, name: str):
    """{short kernel name: [per-dispatch values]} for one counter, plus the calibration kernels."""
    per = collections.defaultdict(list)
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != name:
                    continue
                k = r["Kernel_Name"]
                if "FillFunctor" in k:
                    key = "calibration_fill"
                elif "reduce_kernel" in k and "sum_functor" in k:
                    key = "calibration_sum"
                elif OURS.search(k):
                    key = short_name(k)
                else:
                    continue
                per[key].append(float(r["Counter_Value"]))
    return per


def counters(fetch_dir: str, write_dir: str, out: str, workload: str, command: str) -> None:
    fetch = _counter(fetch_dir, "FETCH_SIZE")
    write = _counter(write_dir, "WRITE_SIZE")
    if "calibration_sum" not in fetch or "calibration_fill" not in write:
        raise SystemExit("calibration kernels missing: run bench.py with --copy-calibration")
    # FETCH_SIZE / WRITE_SIZE are KiB per dispatch
    f_cal = CAL_BYTES / (1024.0 * max(fetch["calibration_sum"]))
    w_cal = CAL_BYTES / (1024.0 * max(write["calibration_fill"]))
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        if k.startswith("calibration"):
            continue
        fv, wv = fetch.get(k, []), write.get(k, [])
        f_avg = sum(fv) / len(fv) if fv else 0.0
        w_avg = sum(wv) / len(wv) if wv else 0.0
        kernels[k] = {
            "dispatches": max(len(fv), len(wv)),
            "fetch_kib_raw": f_avg, "write_kib_raw": w_avg,
            "hbm_bytes_per_launch": 1024.0 * (f_avg * f_cal + w_avg * w_cal),
        }
    # bench.py looks kernels up by their template name without arguments; each
    # carries the hash of the sources that define it
    by_family = {}
    for k, v in kernels.items():
        fam = k.split("<")[0]
        by_family.setdefault(fam, dict(v, source_hash=source_hash(fam)))
    rec = {"workload": workload, "source_hash": source_hash(), "command": command,
           "fetch_factor": f_cal, "write_factor": w_cal,
           "calibration": "fill of 1 GiB (WRITE_SIZE) and sum over 1 GiB (FETCH_SIZE)",
           "kernels": by_family, "kernels_full": kernels}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    b = sub.add_parser("counters")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--workload", required=True)
    b.add_argument("--command", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.dir, args.out, args.command)
    else:
        counters(args.fetch_dir, args.write_dir, args.out, args.workload, args.command)


if __name__ == "__main__":
    main()
