"""Summaries of rocprofv3 output for the roofline of a kernel.

HBM traffic of a kernel comes from two counter runs, `rocprofv3 --pmc
FETCH_SIZE` and `rocprofv3 --pmc WRITE_SIZE` (KiB per dispatch), each scaled
by what the same counter reads for the plain copy kernel `stream_copy_kernel`
of a known size in the same run, so that the counter's unit and any
systematic offset cancel.  Durations come from `rocprofv3 --kernel-trace
--stats`.  The summary is a short text file (key: value lines) that records
the commands, the figures, and a hash of the kernel's sources; a reader of
the summary (the benchmark) uses the traffic only while the hash still
matches the sources.

    python -m paper_1410_5561_amd.profiling --trace DIR --fetch DIR --write DIR \\
        --kernel mwd_row_kernel --workload NAME --dtype f64 --shape 8x64 \\
        --model-bytes-per-launch B --copy-bytes N --out profiles/FILE.txt \\
        --cmd-trace "..." --cmd-fetch "..." --cmd-write "..."

SQ-counter summaries (instruction mix, wait fractions, LDS bank conflicts, L2
hit rate) of one kernel from one or more `rocprofv3 --pmc` runs:

    python -m paper_1410_5561_amd.profiling sq --pmc DIR [DIR ...] --kernel K \\
        --workload NAME --dtype f32 --shape naive --cmd "..." [--cmd "..."] --out FILE
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
PROFILES = os.path.join(ROOT, "profiles")

# sources that decide what a kernel does and how it is compiled
_KERNEL_SOURCES = {
    "mwd_row_kernel": ["mwd_tile.hpp", "mwd_rows.hpp", "common.hpp", "internal.hpp", "mwd.hip",
                       "mwd_inst_7c_f64.hip", "mwd_inst_7c_f32.hip", "mwd_inst_7v_f64.hip",
                       "mwd_inst_7v_f32.hip", "mwd_inst_25c_f64.hip", "mwd_inst_25c_f32.hip",
                       "mwd_inst_25v_f64.hip", "mwd_inst_25v_f32.hip"],
    "naive_sweep_kernel": ["naive.hip", "naive_block.hpp", "common.hpp", "internal.hpp"],
}


def source_hash(kernel: str) -> str:
    """Hash of the sources and compile flags of a kernel family."""
    from . import build as _b
    h = hashlib.sha256()
    h.update(" ".join(_b.CFLAGS).encode())
    for name in _KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _csvs(d, suffix):
    """The run's file of this kind: a directory must hold exactly one run
    (one process), so that runs of different builds are never averaged."""
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if len(files) > 1:
        raise SystemExit("%s holds %d runs (%s files); use a fresh directory per run" % (d, len(files), suffix))
    return files


def kernel_durations(trace_dir, match):
    """(dispatches, average duration in us) of the kernels whose name
    contains `match`, from a --kernel-trace run."""
    n, tot = 0, 0.0
    for p in _csvs(trace_dir, "kernel_trace.csv"):
        with open(p, newline="") as f:
            for r in csv.DictReader(f):
                if match in r.get("Kernel_Name", ""):
                    n += 1
                    tot += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    return n, (tot / n if n else float("nan"))


def kernel_stats_row(trace_dir, match):
    """The --stats line(s) of the kernels whose name contains `match`."""
    rows = []
    for p in _csvs(trace_dir, "kernel_stats.csv"):
        with open(p, newline="") as f:
            for r in csv.DictReader(f):
                if match in r.get("Name", ""):
                    rows.append(r)
    return rows


def counter_per_dispatch(pmc_dir, match, counter):
    """(dispatches, average value) of `counter` over the dispatches of the
    kernels whose name contains `match`, from a --pmc run."""
    per = defaultdict(float)
    for p in _csvs(pmc_dir, "counter_collection.csv"):
        with open(p, newline="") as f:
            for r in csv.DictReader(f):
                if match in r.get("Kernel_Name", "") and r.get("Counter_Name") == counter:
                    per[(p, r["Dispatch_Id"])] += float(r["Counter_Value"])
    n = len(per)
    return n, (sum(per.values()) / n if n else float("nan"))


def read_summary(path):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def summary_path(kernel, workload, dtype, shape):
    name = re.sub(r"[^A-Za-z0-9_.-]", "_", "%s_%s_%s_%s" % (kernel, workload, dtype, shape))
    return os.path.join(PROFILES, name + ".txt")


def traffic_for(kernel, workload, dtype, shape):
    """Measured HBM bytes per launch from a committed summary, or None when
    there is none or the kernel's sources changed since it was taken."""
    p = summary_path(kernel, workload, dtype, shape)
    if not os.path.exists(p):
        return None
    s = read_summary(p)
    if s.get("source_hash") != source_hash(kernel) or "traffic_bytes_per_launch" not in s:
        return None
    return float(s["traffic_bytes_per_launch"])


def sq_counters(pmc_dirs, match):
    """{counter: average per dispatch} over every --pmc run directory given,
    for the kernels whose name contains `match`; and the dispatch count."""
    vals, ndisp = {}, 0
    for d in pmc_dirs:
        per = defaultdict(lambda: defaultdict(float))
        for p in _csvs(d, "counter_collection.csv"):
            with open(p, newline="") as f:
                for r in csv.DictReader(f):
                    if match in r.get("Kernel_Name", ""):
                        per[r["Counter_Name"]][(p, r["Dispatch_Id"])] += float(r["Counter_Value"])
        for c, dd in per.items():
            vals[c] = sum(dd.values()) / len(dd)
            ndisp = max(ndisp, len(dd))
    return vals, ndisp


def sq_summary_lines(vals, ndisp, kernel, workload, dtype, shape, cmds):
    """Key: value lines of an SQ-counter summary with the derived ratios."""
    lines = ["# rocprofv3 SQ counters: %s, workload %s, %s, shape %s" % (kernel, workload, dtype, shape)]
    lines += ["# run: %s" % c for c in cmds]
    lines += ["# values are averages per dispatch of the kernel; wave-cycles are summed over waves",
              "kernel: %s" % kernel, "workload: %s" % workload, "dtype: %s" % dtype, "shape: %s" % shape,
              "source_hash: %s" % source_hash(kernel), "dispatches: %d" % ndisp]
    for c in sorted(vals):
        lines.append("%s: %.1f" % (c, vals[c]))

    def ratio(name, num, den):
        if num in vals and den in vals and vals[den]:
            lines.append("%s: %.4f" % (name, vals[num] / vals[den]))

    ratio("wait_inst_any_over_wave_cycles", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")
    ratio("wait_any_over_wave_cycles", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES")
    ratio("lds_bank_conflict_over_lds_active", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS")
    if "TCC_HIT_sum" in vals and "TCC_MISS_sum" in vals:
        tot = vals["TCC_HIT_sum"] + vals["TCC_MISS_sum"]
        if tot:
            lines.append("l2_hit_rate: %.4f" % (vals["TCC_HIT_sum"] / tot))
    if vals.get("SQ_WAVES"):
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"):
            if c in vals:
                lines.append("%s_per_wave: %.1f" % (c.lower(), vals[c] / vals["SQ_WAVES"]))
    return lines


def sq_main(argv):
    ap = argparse.ArgumentParser(description="Summary of SQ (and L2) counter runs of one kernel.")
    ap.add_argument("--pmc", nargs="+", required=True, help="one directory per rocprofv3 --pmc run")
    ap.add_argument("--kernel", required=True, choices=sorted(_KERNEL_SOURCES))
    ap.add_argument("--workload", required=True)
    ap.add_argument("--dtype", required=True)
    ap.add_argument("--shape", required=True)
    ap.add_argument("--cmd", action="append", required=True, help="the command of each run, in order")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    vals, ndisp = sq_counters(a.pmc, a.kernel)
    lines = sq_summary_lines(vals, ndisp, a.kernel, a.workload, a.dtype, a.shape, a.cmd)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "sq":
        return sq_main(argv[1:])
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True, choices=sorted(_KERNEL_SOURCES))
    ap.add_argument("--workload", required=True)
    ap.add_argument("--dtype", required=True)
    ap.add_argument("--shape", required=True, help="DWxLANES, or naive")
    ap.add_argument("--model-bytes-per-launch", type=float, required=True)
    ap.add_argument("--copy-bytes", type=float, required=True, help="bytes read (= written) per copy dispatch")
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--cmd-fetch", required=True)
    ap.add_argument("--cmd-write", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    nd, avg_us = kernel_durations(a.trace, a.kernel)
    nf, fetch_kib = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    nw, write_kib = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    ncf, copy_fetch_kib = counter_per_dispatch(a.fetch, "stream_copy_kernel", "FETCH_SIZE")
    ncw, copy_write_kib = counter_per_dispatch(a.write, "stream_copy_kernel", "WRITE_SIZE")
    fscale = a.copy_bytes / copy_fetch_kib
    wscale = a.copy_bytes / copy_write_kib
    fetch_b = fetch_kib * fscale
    write_b = write_kib * wscale
    traffic = fetch_b + write_b
    stats = kernel_stats_row(a.trace, a.kernel)
    lines = [
        "# rocprofv3 summary: %s, workload %s, %s, shape %s" % (a.kernel, a.workload, a.dtype, a.shape),
        "# durations: %s" % a.cmd_trace,
        "# FETCH_SIZE: %s" % a.cmd_fetch,
        "# WRITE_SIZE: %s" % a.cmd_write,
        "# Counters are KiB per dispatch; each is scaled by bytes / counter of the copy kernel",
        "# (stream_copy_kernel, %d bytes read and written per dispatch) in the same run." % a.copy_bytes,
        "kernel: %s" % a.kernel,
        "workload: %s" % a.workload,
        "dtype: %s" % a.dtype,
        "shape: %s" % a.shape,
        "source_hash: %s" % source_hash(a.kernel),
        "dispatches_traced: %d" % nd,
        "avg_duration_us: %.2f" % avg_us,
        "dispatches_fetch: %d" % nf,
        "fetch_kib_per_dispatch: %.1f" % fetch_kib,
        "dispatches_write: %d" % nw,
        "write_kib_per_dispatch: %.1f" % write_kib,
        "copy_fetch_kib_per_dispatch: %.1f (%d dispatches)" % (copy_fetch_kib, ncf),
        "copy_write_kib_per_dispatch: %.1f (%d dispatches)" % (copy_write_kib, ncw),
        "fetch_scale_bytes_per_kib: %.2f" % fscale,
        "write_scale_bytes_per_kib: %.2f" % wscale,
        "fetch_bytes_per_launch: %.0f" % fetch_b,
        "write_bytes_per_launch: %.0f" % write_b,
        "traffic_bytes_per_launch: %.0f" % traffic,
        "model_bytes_per_launch: %.0f" % a.model_bytes_per_launch,
        "traffic_over_model: %.3f" % (traffic / a.model_bytes_per_launch),
        "hbm_GBs_at_traffic: %.1f" % (traffic / (avg_us * 1e-6) / 1e9),
    ]
    for r in stats:
        lines.append("# stats: %s calls=%s avg_ns=%s min_ns=%s max_ns=%s" % (
            r.get("Name", "")[:90], r.get("Calls"), r.get("AverageNs"), r.get("MinNs"), r.get("MaxNs")))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
