"""Summarise rocprofv3 CSV output into the short text files kept under profiles/.

  python -m paper_0812_2801_amd.profsum stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_0812_2801_amd.profsum traffic <fetch_dir> <write_dir> <copy_fetch_dir> \
        <copy_write_dir> <copy_bytes> <out.json> "<command>"
  python -m paper_0812_2801_amd.profsum mfma <pmc_dir> <kernel substring> <n_simd> <out.md> "<command>"

`mfma` reports, for the kernels whose name contains the substring, the MFMA
busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs) and the
bf16 MFMA rate (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512 flop over the dispatch
time) against the 2.5 PFLOP/s dense bf16 peak.

`traffic` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the Horner
stage stencil launches by what the same counters read for a plain device copy
of known size, and records the hash of the stencil source they belong to.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STENCIL_SRC = os.path.join(HERE, "csrc", "stencil.hip")

HORNER_MODES = ("1", "2")       # template MODE of the Horner stages (HORNER, HORNER_FIRST)


def is_horner_stage(name: str) -> bool:
    """A Horner-stage launch of one of the stencil kernels (single system,
    x-tiled, batched); the MODE argument is the one before the NORM flag."""
    if not any(k in name for k in ("stencil_kernel<", "stencil_xt_kernel<", "stencil_py_kernel<")):
        return False
    args = name.split("<", 1)[1].split(">", 1)[0].split(",")
    args = [a.strip() for a in args]
    if "batch_stencil_kernel<" in name:          # <T, HJ, MODE, NORM, XT>
        return len(args) >= 3 and args[2] in HORNER_MODES
    return len(args) >= 2 and args[-2] in HORNER_MODES   # <T, ..., MODE, NORM>


def stencil_hash() -> str:
    with open(STENCIL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _counter_rows(d):
    path = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    return list(csv.DictReader(open(path)))


def stats(csv_path, out, command):
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | avg µs | total % |", "|---|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        name = _short(r["Name"]).replace("|", "/")
        if name.startswith("Cijk_") and len(name) > 60:        # library GEMM: tile and MFMA fields only
            name = "_".join(name.split("_")[:6]) + "_..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{100 * float(r['TotalDurationNs']) / tot:.1f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _short(name: str) -> str:
    """Kernel name without its argument list (anonymous namespaces dropped)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0]


def traffic(fetch_dir, write_dir, cf_dir, cw_dir, copy_bytes, out, command):
    def per_kernel(d, pred):
        agg = collections.defaultdict(list)
        for r in _counter_rows(d):
            if pred(r["Kernel_Name"]):
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg

    is_stage = is_horner_stage
    is_copy = lambda k: "copyBuffer" in k
    f = per_kernel(fetch_dir, is_stage)
    w = per_kernel(write_dir, is_stage)
    cf = [v for vs in per_kernel(cf_dir, is_copy).values() for v in vs if v > 1e5]
    cw = [v for vs in per_kernel(cw_dir, is_copy).values() for v in vs if v > 1e5]
    half = copy_bytes / 2.0                  # a copy reads and writes half of it each
    kf = half / (statistics.mean(cf) * 1024.0)
    kw = half / (statistics.mean(cw) * 1024.0)
    fetch = [v for vs in f.values() for v in vs]
    write = [v for vs in w.values() for v in vs]
    per_launch = (statistics.mean(fetch) * kf + statistics.mean(write) * kw) * 1024.0
    res = {"kernel": "stencil_kernel (Horner stages, all launches of the run)",
           "command": command,
           "launches": len(fetch),
           "fetch_scale": kf, "write_scale": kw,
           "fetch_bytes_per_launch": statistics.mean(fetch) * kf * 1024.0,
           "write_bytes_per_launch": statistics.mean(write) * kw * 1024.0,
           "bytes_per_launch": per_launch,
           "by_kernel": {_short(k): {"fetch_KiB": statistics.mean(v),
                                            "write_KiB": statistics.mean(w.get(k, [0.0]))}
                         for k, v in f.items()},
           "stencil_sha256_16": stencil_hash()}
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def mfma(pmc_dir, pattern, n_simd, out, command):
    per = collections.defaultdict(dict)
    names = {}
    for r in _counter_rows(pmc_dir):
        if pattern not in r["Kernel_Name"]:
            continue
        d = r["Dispatch_Id"]
        per[d][r["Counter_Name"]] = per[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        per[d]["ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        names[d] = _short(r["Kernel_Name"])
    util, rate, dur = [], [], []
    for d, c in per.items():
        util.append(100.0 * c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] * n_simd))
        rate.append(c["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0 / (c["ns"] * 1e-9) / 1e12)
        dur.append(c["ns"] / 1e3)
    kname = sorted(set(names.values()))
    lines = ["# MFMA use of the split-bf16 projector contraction", "", f"Command: `{command}`", "",
             f"Kernels: {', '.join('`' + k + '`' for k in kname)}; {len(util)} dispatches.", "",
             "| quantity | mean | min | max |", "|---|---:|---:|---:|",
             f"| duration (µs) | {statistics.mean(dur):.2f} | {min(dur):.2f} | {max(dur):.2f} |",
             f"| MFMA busy (% of SIMD cycles) | {statistics.mean(util):.3f} | {min(util):.3f} | {max(util):.3f} |",
             f"| bf16 MFMA rate (TFLOP/s) | {statistics.mean(rate):.3f} | {min(rate):.3f} | {max(rate):.3f} |",
             f"| fraction of the 2.5 PFLOP/s dense bf16 peak (%) | {100 * statistics.mean(rate) / 2500:.4f} | | |"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], float(sys.argv[6]), sys.argv[7],
                sys.argv[8])
    elif sys.argv[1] == "mfma":
        mfma(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
