"""Condense rocprofv3 output into the short summaries kept under profiles/.

    # kernel durations (rocprofv3 --kernel-trace --stats ... --output-format csv)
    python -m paper_1803_00005_amd.profile_summary stats DIR OUT.md --command "..."

    # HBM bytes per launch from two counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE)
    python -m paper_1803_00005_amd.profile_summary counters FETCH_DIR WRITE_DIR OUT.json \
        --workload NAME --command "..."

    # VALU, LDS, wave-occupancy and L2 counters (one or more --pmc runs)
    python -m paper_1803_00005_amd.profile_summary units OUT.md DIR [DIR ...] \
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
    k = k.split("hgf::")[-1] if "hgf::" in k else k[:60]
    # kernels in the library's inner namespaces keep their plain names
    for ns in ("gk::", "sk::"):
        if k.startswith(ns):
            k = k[len(ns):]
    return k


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


SIMDS = 256 * 4   # MI355X: 256 CUs of 4 SIMDs


def _all_counters(dirs):
    """{short kernel name: {counter: mean value per dispatch}} over the runs' files."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for f in _find(d, "counter_collection.csv"):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if not OURS.search(r["Kernel_Name"]):
                        continue
                    acc[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(
                        float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


XCDS = 8          # GRBM_GUI_ACTIVE is counted once per XCD


def units(out: str, dirs, workload: str, command: str) -> None:
    """Per-kernel VALU, LDS, occupancy and L2 figures from raw SQ/TCC/GRBM counters.

    cycles       = GRBM_GUI_ACTIVE / 8 (the counter is summed over the 8 XCDs;
                   cycles / clock reproduces the kernel's duration)
    VALU busy    = 4 * SQ_INSTS_VALU / (SIMDs * cycles): the share of SIMD cycles
                   spent issuing vector ALU instructions (a wave64 instruction
                   occupies a SIMD for 4 cycles without packed FP32)
    VALU / wave  = SQ_INSTS_VALU / SQ_WAVES
    LDS / wave   = SQ_INSTS_LDS / SQ_WAVES
    LDS conflict = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS
    waves / CU   = 4 * SQ_WAVE_CYCLES / cycles / 256 (mean resident waves per CU;
                   SQ_WAVE_CYCLES counts wave residency in units of four cycles,
                   summed over the CUs)
    L2 hit       = TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)
    """
    data = _all_counters(dirs)
    lines = ["# Vector ALU, LDS, occupancy and L2 counters", "",
             f"Workload: `{workload}`.  Commands (from the repository root on the GPU "
             "machine, one run per counter group):", "", "```", command, "```", "",
             "Derived: cycles = GRBM_GUI_ACTIVE / 8 (one count per XCD); VALU busy = "
             "4 SQ_INSTS_VALU / (1024 SIMDs x cycles); waves / CU = 4 SQ_WAVE_CYCLES / "
             "cycles / 256; L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS).", "",
             "| kernel | cycles | VALU busy | VALU instr / wave | LDS instr / wave | LDS bank "
             "conflicts / LDS cycle | mean waves / CU | L2 hit |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]

    def g(c, k, default=None):
        return c.get(k, default)

    raw = {}
    for k in sorted(data, key=lambda k: -data[k].get("GRBM_GUI_ACTIVE", 0.0)):
        c = data[k]
        cyc = busy = vpw = lpw = conf = occ = hit = None
        if g(c, "GRBM_GUI_ACTIVE"):
            cyc = c["GRBM_GUI_ACTIVE"] / XCDS
        if g(c, "SQ_INSTS_VALU") and cyc:
            busy = 4 * c["SQ_INSTS_VALU"] / SIMDS / cyc
        if g(c, "SQ_INSTS_VALU") and g(c, "SQ_WAVES"):
            vpw = c["SQ_INSTS_VALU"] / c["SQ_WAVES"]
        if g(c, "SQ_INSTS_LDS") is not None and g(c, "SQ_WAVES"):
            lpw = c["SQ_INSTS_LDS"] / c["SQ_WAVES"]
        if g(c, "SQ_LDS_BANK_CONFLICT") is not None and g(c, "SQ_ACTIVE_INST_LDS"):
            conf = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_ACTIVE_INST_LDS"]
        if g(c, "SQ_WAVE_CYCLES") and cyc:
            occ = 4 * c["SQ_WAVE_CYCLES"] / cyc / 256
        h, m = g(c, "TCC_HIT_sum"), g(c, "TCC_MISS_sum")
        if h is not None and m is not None and h + m > 0:
            hit = h / (h + m)

        def f(v, fmt):
            return "n/a" if v is None else format(v, fmt)

        lines.append(f"| `{k}` | {f(cyc, '.0f')} | {f(busy, '.1%')} | {f(vpw, '.0f')} | "
                     f"{f(lpw, '.0f')} | {f(conf, '.3f')} | {f(occ, '.1f')} | {f(hit, '.1%')} |")
        raw[k] = c
    lines += ["", "Raw counters (mean per dispatch):", "", "```",
              json.dumps(raw, indent=1, sort_keys=True), "```", "",
              f"Kernel sources: `{source_hash()}`", ""]
    with open(out, "w") as fh:
        fh.write("\n".join(lines))


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
    c = sub.add_parser("units")
    c.add_argument("out")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--workload", required=True)
    c.add_argument("--command", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.dir, args.out, args.command)
    elif args.cmd == "counters":
        counters(args.fetch_dir, args.write_dir, args.out, args.workload, args.command)
    else:
        units(args.out, args.dirs, args.workload, args.command)


if __name__ == "__main__":
    main()
