"""Counter bookkeeping for the roofline report.

``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` (two separate runs of
``bench.py --copy-calib-mib N``) give, per dispatch, the HBM-side read and
write volume in KiB.  The same runs include a plain device copy of N MiB,
whose readings fix the scale between counter units and bytes on this chip.
``summarize`` turns the two counter CSVs into a small text record (kept under
``profiles/``) holding the bytes per launch of one kernel and a hash of the
kernel sources; ``load_traffic`` returns those bytes only while the sources
still hash the same, so a stale measurement is never reported.

``trace_summary`` turns a ``rocprofv3 --kernel-trace --stats`` run into a
short markdown summary: the per-kernel statistics of the whole run, the mean
duration of the last ``LAST`` dispatches of each named kernel (the held
repetitions bench.py times, which its ``avg_launch_us`` must match), and
selected fields of the bench line.

Usage:
    python -m paper_2307_03307_amd.profiling FETCH_DIR WRITE_DIR KERNEL COPY_MIB OUT [LAST]
    python -m paper_2307_03307_amd.profiling trace TRACE_DIR TITLE COMMAND OUT BENCH_JSON LAST KERNEL...
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources whose text defines each kernel family and its data layout (shared
# helpers, the kernels, and the host program that lays out the device arrays)
KERNEL_SOURCES = {"vc_": ["device_common.h", "vcover.hip", "program_vcover.cpp"],
                  "k_": ["device_common.h", "generic.hip", "program_generic.cpp"],
                  "kb_": ["device_common.h", "batch.hip", "program_batch.cpp"],
                  "dn_": ["device_common.h", "densest.hip", "program_densest.cpp"]}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash(kernel: str) -> str:
    """Hash of the sources of `kernel`'s family (by name prefix)."""
    files = next(v for k, v in KERNEL_SOURCES.items() if kernel.startswith(k))
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(d: str, counter: str):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    out.sort()
    return out


def _kernel_values(rows, kernel: str, last: int):
    vals = [v for _, k, v in rows if kernel in k]
    return vals[-last:] if last else vals


def summarize(fetch_dir: str, write_dir: str, kernel: str, copy_mib: int, last: int = 10) -> dict:
    """Bytes per launch of `kernel` (mean over its last `last` dispatches, the
    timed repetitions of bench.py) scaled by the copy calibration."""
    copy_bytes = copy_mib * float(1 << 20)
    rec = {"kernel": kernel, "source_sha": source_hash(kernel), "copy_mib": copy_mib}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _rows(d, counter)
        copies = [v for _, k, v in rows if COPY_KERNEL in k]
        big = max(copies) if copies else 0.0
        factor = copy_bytes / (big * 1024.0) if big > 0 else float("nan")
        vals = _kernel_values(rows, kernel, last)
        kib = statistics.mean(vals) if vals else float("nan")
        rec[f"{name}_kib_raw"] = kib
        rec[f"{name}_copy_kib_raw"] = big
        rec[f"{name}_factor"] = factor
        rec[f"{name}_bytes"] = kib * 1024.0 * factor
        rec[f"{name}_dispatches"] = len(vals)
    rec["traffic_bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
    return rec


def write_record(rec: dict, path: str, command: str) -> None:
    with open(path, "w") as f:
        f.write(f"# HBM traffic per launch of {rec['kernel']} (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n")
        f.write(f"# command: {command}\n")
        for k, v in rec.items():
            f.write(f"{k}: {v}\n")


def load_traffic(path: str, kernel: str):
    """traffic_bytes of the record at `path` if it covers `kernel` and the
    kernel sources have not changed since it was taken, else None."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel") != kernel or rec.get("source_sha") != source_hash(kernel):
        return None
    try:
        return float(rec["traffic_bytes"])
    except (KeyError, ValueError):
        return None


BENCH_KEYS = ("value", "unit", "fp64_plain_s", "speedup_vs_fp64", "iterations", "fp64_iterations",
              "certified", "roofline", "passes", "fp64_batched_s", "fp64_loop_s", "speedup_vs_fp64_loop",
              "speedup_vs_fp64_batched", "exact_optimum_in_bracket", "layout", "tuned_layout_s", "passes_full_list")


def trace_summary(trace_dir: str, title: str, command: str, out: str, bench_json: str, last: int,
                  kernels) -> None:
    import json
    stats = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(stats[0])))
    held = {}
    traces = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if traces and kernels:
        disp = []
        with open(traces[0]) as fh:
            for r in csv.DictReader(fh):
                disp.append((int(r["Start_Timestamp"]), r["Kernel_Name"],
                             int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        disp.sort()
        for k in kernels:
            d = [ns for _, n, ns in disp if k in n]
            if d:
                held[k] = statistics.mean(d[-last:]) / 1e3
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommand (run from the repository root on one MI355X):\n\n```\n{command}\n```\n\n")
        f.write("rocprofv3 kernel statistics of the whole run (every dispatch, including no-op launches\n"
                "of kernels whose phase was inactive in a captured iteration slot, passes over the\n"
                "full lists before the active lists exist, and the held timing repetitions):\n\n")
        f.write("| kernel | calls | avg us | total ms | % |\n|---|---:|---:|---:|---:|\n")
        for r in rows[:30]:
            name = r["Name"].split("(")[0].replace("void ", "").replace("mwu::", "")
            f.write(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.2f} |\n")
        if held:
            f.write(f"\nMean duration of the last {last} dispatches (the held repetitions bench.py times):\n\n")
            for k, v in held.items():
                f.write(f"- `{k}`: {v:.2f} us\n")
        if bench_json and os.path.exists(bench_json):
            d = json.loads(open(bench_json).read().strip().splitlines()[-1])
            keep = {k: d[k] for k in BENCH_KEYS if k in d}
            f.write("\nBench line of the same run (selected fields):\n\n```\n" + json.dumps(keep, indent=1) + "\n```\n")


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "trace":
    trace_dir, title, command, out, bench_json, last = sys.argv[2:8]
    trace_summary(trace_dir, title, command, out, bench_json, int(last), sys.argv[8:])
elif __name__ == "__main__":
    fetch_dir, write_dir, kernel, copy_mib, out = sys.argv[1:6]
    last = int(sys.argv[6]) if len(sys.argv) > 6 else 10
    r = summarize(fetch_dir, write_dir, kernel, int(copy_mib), last)
    cmd = os.environ.get("PMC_COMMAND", "bench.py --copy-calib-mib " + copy_mib)
    write_record(r, out, cmd)
    print(r)
