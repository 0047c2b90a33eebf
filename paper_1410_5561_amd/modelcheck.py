"""Memory-traffic model against measured HBM traffic, per tile shape (the GPU
counterpart of the paper's model validation, Sec. III-B, III-C and IV-B,
Fig. 3).

For each tile shape (diamond width Dw and x lanes, or the naive sweep) of
one workload, two rocprofv3 counter runs of one whole run (``bench.py
--steps 1 --warmup 0``) give FETCH_SIZE and WRITE_SIZE per dispatch; each is
scaled by what the same counter reads for the streaming copy of known size
in the same run (as in ``profiling``), summed over the run's dispatches of
the stencil kernels, and divided by the run's lattice-site updates.  The
model is Eq. (5), 2 s R ((2 Dw - 2R) + (N_D Dw + 2R)) / Dw^2 bytes per
update (s N_D for the naive sweep).  The paper's Eq. (3) gives the cache
block a wavefront needs on a CPU; on the GPU the tile's working set is held
in LDS (the exchange planes) and in registers (z-queues, coefficient ring,
prefetch rings); the counter runs report the LDS size, the workgroup size
and the register spill (scratch) per kernel.

    python -m paper_1410_5561_amd.modelcheck --root DIR --workload NAME \\
        --kind 7v --dtype f64 --lups-per-run N --copy-bytes B --out profiles/FILE.txt \\
        --cmd "..." SHAPE [SHAPE ...]

Each SHAPE is DWxLANES (or "naive") and names the subdirectories
DIR/SHAPE/fetch and DIR/SHAPE/write.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
from collections import defaultdict

ND = {"7c": 2, "7v": 9, "25c": 2, "25v": 15}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}
KERNELS = ("mwd_row_kernel", "naive_sweep_kernel", "mwd_gather_kernel", "mwd_halo_fill_kernel")


def model_bytes_per_lup(kind, elem, dw):
    R, n = RADIUS[kind], ND[kind]
    if dw == 0:
        return elem * n
    return 2.0 * elem * R * ((2 * dw - 2 * R) + (n * dw + 2 * R)) / (dw * dw)


def _rows(d):
    """Rows of the run's counter file (one process: one whole run)."""
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if len(files) != 1:
        raise SystemExit("expected one counter file under %s, found %d" % (d, len(files)))
    with open(files[0], newline="") as f:
        for r in csv.DictReader(f):
            yield files[0], r


def counter_sums(d, counter):
    """{kernel family: (dispatches, summed value)} and the copy kernel's
    average, for one counter run; plus per-family resource columns."""
    per = defaultdict(float)
    kern = {}
    res = {}
    for p, r in _rows(d):
        if r.get("Counter_Name") != counter:
            continue
        key = (p, r["Dispatch_Id"])
        per[key] += float(r["Counter_Value"])
        kern[key] = r.get("Kernel_Name", "")
        fam = next((k for k in KERNELS + ("stream_copy_kernel",) if k in kern[key]), None)
        if fam and fam not in res:
            res[fam] = {c: r.get(c) for c in ("VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
                                              "LDS_Block_Size", "Scratch_Size", "Workgroup_Size")}
    sums = defaultdict(lambda: [0, 0.0])
    for key, v in per.items():
        fam = next((k for k in KERNELS + ("stream_copy_kernel",) if k in kern[key]), "other")
        sums[fam][0] += 1
        sums[fam][1] += v
    return sums, res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--root", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kind", required=True, choices=sorted(ND))
    ap.add_argument("--dtype", required=True, choices=("f64", "f32"))
    ap.add_argument("--lups-per-run", type=float, required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--cmd", required=True, help="the command of one counter run, with SHAPE and COUNTER")
    ap.add_argument("--out", required=True)
    ap.add_argument("shapes", nargs="+")
    a = ap.parse_args(argv)
    elem = 8 if a.dtype == "f64" else 4
    lines = [
        "# Measured HBM traffic against the Eq. (5) model, workload %s (%s %s)" % (a.workload, a.kind, a.dtype),
        "# counter runs: %s" % a.cmd,
        "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the copy kernel's reading of",
        "# %d bytes per dispatch in the same run; summed over one whole run; per lattice-site update" % a.copy_bytes,
        "# (%d updates per run).  tile = stencil kernels only (row kernels or naive sweeps);" % a.lups_per_run,
        "# all = also the boundary fill and the final gather of the MWD schedule.",
        "# on-chip: LDS bytes and threads per workgroup, register-spill (scratch) bytes per lane.",
        "%-8s %9s %9s %9s %7s %7s  %s" % ("shape", "model", "tile", "all", "t/m", "a/m", "on-chip"),
    ]
    for shape in a.shapes:
        dw = 0 if shape == "naive" else int(shape.split("x")[0])
        model = model_bytes_per_lup(a.kind, elem, dw)
        tot = {}
        resources = {}
        for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
            sums, res = counter_sums(os.path.join(a.root, shape, sub), counter)
            resources.update(res)
            nc, cv = sums.get("stream_copy_kernel", [0, 0.0])
            if nc == 0 or cv == 0:
                raise SystemExit("no copy kernel in %s/%s" % (shape, sub))
            scale = a.copy_bytes / (cv / nc)
            tile = sum(sums[k][1] for k in ("mwd_row_kernel", "naive_sweep_kernel") if k in sums) * scale
            allk = sum(sums[k][1] for k in KERNELS if k in sums) * scale
            tot[sub] = (tile, allk)
        tile_b = (tot["fetch"][0] + tot["write"][0]) / a.lups_per_run
        all_b = (tot["fetch"][1] + tot["write"][1]) / a.lups_per_run
        fam = "naive_sweep_kernel" if dw == 0 else "mwd_row_kernel"
        r = resources.get(fam, {})
        chip = "LDS %s B, workgroup %s, scratch %s B" % (r.get("LDS_Block_Size"), r.get("Workgroup_Size"),
                                                           r.get("Scratch_Size"))
        lines.append("%-8s %9.3f %9.3f %9.3f %7.3f %7.3f  %s" % (shape, model, tile_b, all_b, tile_b / model,
                                                               all_b / model, chip))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
