"""Benchmark: GLUP/s of the MWD-blocked stencil sweep on one MI355X, against the
naive one-sweep-per-step schedule, with the HBM roofline and the CPU oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]
                    [--mode auto|mwd|naive] [--dw D] [--lanes L]

A step is one whole run of the hot path: T time steps of the workload's
stencil over its grid (inputs resident in HBM), i.e. one stencil_run call.
Each step continues from the previous one's result (the two-array state);
values decay slowly (weights sum to <= 1) and stay far from subnormals.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--batch-count", type=int, default=256, help="grids in workload 5")
    ap.add_argument("--dtype", default=None, help="for workload 3: f64 or f32")
    ap.add_argument("--mode", default="auto", choices=["auto", "mwd", "naive"])
    ap.add_argument("--dw", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--naive-steps", type=int, default=2)
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-against-FP64 sub-run of an FP32 workload")
    ap.add_argument("--no-energy", action="store_true",
                    help="skip the GPU energy-to-solution measurement (AMD SMI energy counter)")
    ap.add_argument("--cpu-T", type=int, default=0, help="time steps of the oracle sample")
    ap.add_argument("--sweep", action="store_true",
                    help="also time every compiled MWD shape (diamond width x lanes)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (4 in FP32, 3 in FP64 and FP32, 5) that the "
                         "default line reports beside the headline workload")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of each other workload")
    ap.add_argument("--energy-sweep", action="store_true",
                    help="energy to solution of the naive sweep and every MWD diamond width on the "
                         "workload's grid, in FP64 and FP32 (GPU socket energy counter)")
    ap.add_argument("--kind", default=None, choices=["25v"],
                    help="workload 3 with 13 seeded weight arrays (25-point variable stencil)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the runs with per-launch events (no roofline): for counter runs, "
                         "which then see exactly the timed runs")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def log(a, *msg):
    if a.verbose:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def make_inputs(w, dtype, windex):
    """Seeded inputs of a workload (recipe in gridgen)."""
    import gridgen
    nx, ny, nz = w["n"]
    R = gridgen.RADIUS[w["kind"]]
    seed = gridgen.seed_for_config(windex)
    npdt = np.float64 if dtype == "f64" else np.float32
    u0 = gridgen.field(seed, nx, ny, nz, R, *w["field"], dtype=npdt)
    return u0, workload_coeffs(w, seed, (nx, ny, nz), R, npdt)


def workload_coeffs(w, seed, n, R, npdt):
    """The workload's weights: constants, or the seeded arrays of a variable kind."""
    import gridgen
    if w["coeffs"] == "7v":
        return gridgen.coeffs_7v(seed, *n, R, dtype=npdt)
    if w["coeffs"] == "25v":
        return gridgen.coeffs_25v(seed, *n, R, dtype=npdt)
    return list(w["coeffs"])


def workload(windex, kind=None):
    """Workload windex; kind "25v" turns workload 3 into its variable-weight
    form (same grid, field and T; 13 seeded weight arrays)."""
    import gridgen
    w = dict(gridgen.workloads()[windex])
    if kind:
        if windex != 3 or kind != "25v":
            raise SystemExit("--kind 25v applies to workload 3 only")
        w.update(kind="25v", coeffs="25v", name="25v-512^3-T32")
    return w


KERNEL_TIMING = True


def time_mode(S, torch, kind, dtype, n, u0_dev, co_dev, T, steps, warmup, mode, dw, lanes, halo, meter=None):
    """Run warmup + timed steps; return (seconds, plan description, profile).
    With an energy meter, also the energy of repeated runs (outside the timed
    steps) in desc["energy"]."""
    a = u0_dev.clone()
    b = u0_dev.clone()
    g = S.make_grid(a, b, halo, 0)
    if kind in ("7c", "25c"):
        c = S.make_coeffs(kind, consts=co_dev)
    else:
        c = S.make_coeffs(kind, arrays=co_dev)
    if mode == "auto":
        plan = S.Plan(kind, dtype, *n)
    else:
        plan = S.Plan(kind, dtype, *n, mode=mode, dw=dw, lanes=lanes)
    for _ in range(warmup):
        plan.run(g, c, T)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    t0 = time.perf_counter()
    for i in range(steps):
        plan.run(g, c, T)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = evs[0].elapsed_time(evs[-1]) / 1e3
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    # kernel durations: as many runs again, with the plan's per-launch events
    # (skipped with --no-kernel-timing: counter runs then see one set of runs)
    prof = {"main_ms": 0.0, "main_launches": 0, "other_ms": 0.0, "other_launches": 0}
    if KERNEL_TIMING:
        plan.profile(True)
        plan.profile_read()  # drop anything recorded so far
        for i in range(steps):
            plan.run(g, c, T)
        torch.cuda.synchronize()
        prof = plan.profile_read()
        plan.profile(False)
    desc = plan.describe()
    desc["step_ms"] = {"min": round(per_step[0], 4), "median": round(per_step[len(per_step) // 2], 4),
                       "max": round(per_step[-1], 4)}
    # FP64 norms (on the GPU) of the last level and of the last step's change
    l2, mx = S.stencil_norms(g, 0)
    rl2, rmx = S.stencil_norms(g, 1)
    desc["norms"] = {"u_l2": l2, "u_max": mx, "residual_l2": rl2, "residual_max": rmx}
    if meter is not None and meter.ok:
        from paper_1410_5561_amd import energy
        # three windows of repeated runs; the median window by energy per LUP
        wins = []
        clk = []
        for _ in range(3):
            reps, dt, joules, smu_w = energy.measure(meter, lambda: plan.run(g, c, T), torch.cuda.synchronize,
                                                     min_seconds=1.5,
                                                     on_sync=lambda: clk.append(meter.clocks_mhz()))
            lups = n[0] * n[1] * n[2] * T * reps
            wins.append({"runs": reps, "seconds": round(dt, 3), "joules": round(joules, 3),
                         "avg_power_W": round(joules / dt, 1),
                         "firmware_avg_power_W": None if smu_w is None else round(smu_w, 1),
                         "pJ_per_LUP": round(joules / lups * 1e12, 2),
                         "GLUP_per_s": round(lups / dt / 1e9, 2)})
        wins.sort(key=lambda e: e["pJ_per_LUP"])
        desc["energy"] = dict(wins[1], pJ_per_LUP_windows=[e["pJ_per_LUP"] for e in wins])
        clk = [c for c in clk if c]
        if clk:
            # clocks read at the windows' synchronisations, while the runs load the GPU
            desc["energy"]["sclk_MHz"] = round(sum(c["sclk"] for c in clk) / len(clk))
            desc["energy"]["mclk_MHz"] = round(sum(c["mclk"] for c in clk) / len(clk))
    state = (a, b)[g.cur]
    plan.close()
    return max(ev, 1e-9), wall, desc, prof, state


FLOPS_PER_LUP = {"7c": 10, "7v": 13, "25c": 37, "25v": 37}


def precision_subrun(S, torch, w, windex, n=(256, 256, 256)):
    """The FP32 form against FP64 on a sub-run of the workload (same kind, T
    and seed, an n-point interior), all on the GPU, the difference's norms
    reduced in FP64 on the GPU.  Three runs: FP32 on the casts of the FP64
    draws; FP64 on those same FP32-rounded inputs, widened (the primary
    reference: it isolates the FP32 arithmetic); FP64 on the original draws
    (the error of choosing FP32 at all).  The FP64 runs are the oracle's
    results (bit-exact, as the parity tests check).

    A priori bounds: every weight set here is non-negative with sum <= 1, so
    one sweep does not amplify an error in the max norm and keeps |u| below
    |u0|max; each sweep adds at most ops roundings of unit 2^-24 (ops = the
    flops of one update), plus one on the FP64 side's behalf: T * (ops + 1)
    * 2^-24 * |u0|max.  Against the original draws the FP32 weights add one
    more per sweep and the cast of u0 one in all."""
    import gridgen
    kind, T = w["kind"], w["T"]
    R = gridgen.RADIUS[kind]
    seed = gridgen.seed_for_config(windex)
    u64 = gridgen.field(seed, *n, R, *w["field"], dtype=np.float64)
    c64 = workload_coeffs(w, seed, n, R, np.float64)

    def widened(x):
        return np.asarray(x, dtype=np.float32).astype(np.float64)

    runs = {"f32": ("f32", u64.astype(np.float32),
                    [np.asarray(c, dtype=np.float32) for c in c64]),
            "f64_on_f32_inputs": ("f64", widened(u64), [widened(c) for c in c64]),
            "f64": ("f64", u64, [np.asarray(c, dtype=np.float64) for c in c64])}
    out = {}
    for name, (dt, u0, co) in runs.items():
        a = torch.from_numpy(u0).cuda()
        b = a.clone()
        g = S.make_grid(a, b, R, 0)
        if kind in ("7c", "25c"):
            cdev = None
            c = S.make_coeffs(kind, consts=[float(x) for x in co])
        else:
            cdev = [torch.from_numpy(x).cuda() for x in co]
            c = S.make_coeffs(kind, arrays=cdev)
        plan = S.Plan(kind, dt, *n)
        plan.run(g, c, T)
        torch.cuda.synchronize()
        plan.close()
        out[name] = (g, (a, b), cdev)
    u0max = float(np.max(np.abs(u64)))
    ops = FLOPS_PER_LUP[kind]
    res = {"sub_run": "%s %dx%dx%d T=%d, seed of the workload" % (kind, n[0], n[1], n[2], T)}
    for ref, bound in (("f64_on_f32_inputs", T * (ops + 1) * 2.0 ** -24 * u0max),
                       ("f64", (T * (ops + 2) + 1) * 2.0 ** -24 * u0max)):
        err_l2, err_max = S.stencil_diff_norms(out["f32"][0], out[ref][0])
        ref_l2, ref_max = S.stencil_norms(out[ref][0], 0)
        res["vs_" + ref] = {"max_abs_err": err_max,
                            "max_rel_err": err_max / ref_max if ref_max else err_max,
                            "l2_rel_err": err_l2 / ref_l2 if ref_l2 else err_l2,
                            "a_priori_bound": bound,
                            "within_bound": bool(err_max <= bound and math.isfinite(err_l2))}
    return res


def cpu_baseline(w, dtype, windex, T_cpu, min_s=10.0, max_reps=20):
    """Time the oracle (as it is) on the host cores on a bounded sample."""
    import gridgen
    import oracle
    nx, ny, nz = w["n"]
    R = gridgen.RADIUS[w["kind"]]
    # a sample of the same workload: the full grid, fewer time steps
    u0, co = make_inputs(w, dtype, windex)
    threads = oracle.default_threads()
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    # T_cpu steps at a time, continuing from the last result, until the
    # sample has taken at least min_s seconds (or max_reps repeats)
    t0 = time.perf_counter()
    steps, u = 0, u0
    while True:
        u, _ = oracle.run(w["kind"], u, co, T_cpu, halo=R, threads=threads)
        steps += T_cpu
        dt = time.perf_counter() - t0
        if dt >= min_s or steps >= max_reps * T_cpu:
            break
    lups = nx * ny * nz * steps
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": lups / dt / 1e9, "unit": "GLUP/s", "cores": threads, "kind": "oracle",
            "cpu": cpu, "host_cpus": os.cpu_count(),
            "sample": "%s, full %dx%dx%d grid, %d steps (%d runs of T=%d), %.1f s" % (
                w["kind"] + "-" + dtype, nx, ny, nz, steps, steps // T_cpu, T_cpu, dt)}


def batch_measure(a, torch, S, steps, warmup):
    """Workload 5: many uneven grids (7-point and 25-point constant, FP32)
    advanced together with one hipGraph launch per step.  Returns
    (GLUP/s, seconds of the timed steps, grids, LUPs per step)."""
    import gridgen
    w = gridgen.workloads()[5]
    T = w["T"]
    specs = gridgen.batch_specs(count=a.batch_count)
    log(a, "batch inputs", len(specs))
    grids, keep, coeffs = [], [], []
    lups = 0
    for sp in specs:
        u0 = gridgen.batch_field(sp, np.float32)
        d = torch.from_numpy(u0).cuda()
        keep.append((d, d.clone()))
        grids.append(S.make_grid(keep[-1][0], keep[-1][1], sp["halo"], 0))
        coeffs.append(S.make_coeffs(sp["kind"], consts=sp["coeffs"]))
        nx, ny, nz = sp["n"]
        lups += nx * ny * nz * T
    plan = S.Plan("mixed", "f32")
    for _ in range(max(1, warmup)):
        plan.run_batched(grids, coeffs, T)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.run_batched(grids, coeffs, T)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    plan.close()
    del keep
    return steps * lups / sec / 1e9, sec, len(specs), lups


def bench_batch(a, torch, S):
    """The batching workload as the headline line (--workload 5)."""
    import gridgen
    w = gridgen.workloads()[5]
    T = w["T"]
    value, sec, ngrids, lups = batch_measure(a, torch, S, a.steps, a.warmup)
    # model bytes: each grid at its own Eq. (5) balance would need the tuned
    # shapes; report the naive-sweep balance (s N_D = 8 B/LUP) as the ceiling
    out = {
        "metric": "GLUP/s + rocprof bytes/LUP, MWD vs naive sweep, FP64 and FP32, 1 GPU",
        "value": round(value, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(sec * 1e3 / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "grids": ngrids, "T": T, "lups_per_step": lups},
    }
    print(json.dumps(out), flush=True)
    return 0


def energy_sweep(a, torch, S, windex):
    """Energy to solution per lattice-site update against the code balance:
    the naive sweep and each MWD tile shape, FP64 and FP32, on one workload's
    grid (the counterpart of the energy tables and the energy-vs-code-balance
    figure of Sec. IV-C).  Each point: three windows of >= 1.5 s of repeated
    whole runs; the median window."""
    import gridgen
    from paper_1410_5561_amd import energy
    w = gridgen.workloads()[windex]
    kind, n, T = w["kind"], w["n"], w["T"]
    R = gridgen.RADIUS[kind]
    shapes = {1: [("naive", 0, 0), ("mwd", 4, 64), ("mwd", 4, 128), ("mwd", 4, 256), ("mwd", 8, 64),
                  ("mwd", 8, 128), ("mwd", 10, 64)],
              4: [("naive", 0, 0), ("mwd", 8, 64), ("mwd", 8, 128), ("mwd", 16, 64)]}[R]
    meter = energy.EnergyMeter()
    out = {"workload": w["name"], "meter": "AMD SMI energy counter of the GPU socket", "points": []}
    if not meter.ok:
        out["error"] = meter.error
        return out
    for dtype in ("f64", "f32"):
        u0, co = make_inputs(w, dtype, windex)
        u0_dev = torch.from_numpy(u0).cuda()
        co_dev = co if kind in ("7c", "25c") else [torch.from_numpy(c).cuda() for c in co]
        del u0, co
        for mode, dw, lanes in shapes:
            try:
                sec, _, desc, _, st = time_mode(S, torch, kind, dtype, n, u0_dev, co_dev, T, 2, 1, mode,
                                                dw, lanes, R, meter=meter)
            except Exception as e:  # a shape not compiled for this dtype
                out["points"].append({"dtype": dtype, "mode": mode, "dw": dw, "lanes": lanes,
                                      "error": str(e)[:80]})
                continue
            del st
            en = desc.get("energy") or {}
            out["points"].append({"dtype": dtype, "mode": mode, "dw": dw, "lanes": lanes,
                                  "model_bytes_per_lup": round(desc["model_bytes_per_lup"], 3),
                                  "GLUP_per_s": en.get("GLUP_per_s"), "pJ_per_LUP": en.get("pJ_per_LUP"),
                                  "avg_power_W": en.get("avg_power_W"),
                                  "pJ_per_LUP_windows": en.get("pJ_per_LUP_windows")})
            log(a, "energy point", out["points"][-1])
        del u0_dev, co_dev
        torch.cuda.empty_cache()
    meter.close()
    return out


def other_workload(a, torch, S, windex, dtype):
    """A compact line for one more workload: the autotuned plan against the
    naive sweep, both timed over whole runs with inputs resident."""
    import gridgen
    w = gridgen.workloads()[windex]
    kind, (nx, ny, nz), T = w["kind"], w["n"], w["T"]
    R = gridgen.RADIUS[kind]
    lups = nx * ny * nz * T
    log(a, "other workload", w["name"], dtype)
    u0, co = make_inputs(w, dtype, windex)
    u0_dev = torch.from_numpy(u0).cuda()
    co_dev = co if kind in ("7c", "25c") else [torch.from_numpy(c).cuda() for c in co]
    del u0, co
    steps = a.extra_steps
    sec, _, desc, prof, state = time_mode(S, torch, kind, dtype, (nx, ny, nz), u0_dev, co_dev, T,
                                          steps, 1, "auto", 0, 0, R)
    del state
    value = steps * lups / sec / 1e9
    mode_name = {0: "auto", 1: "naive", 2: "mwd"}[desc["mode"]]
    bpl = desc["model_bytes_per_lup"]
    launches = max(1, prof["main_launches"])
    achieved = bpl * lups * steps / launches / (prof["main_ms"] / 1e3 / launches) / 1e9 if prof["main_ms"] else 0.0
    res = {"workload": w["name"], "dtype": dtype, "value": round(value, 3), "unit": "GLUP/s",
           "steps": steps, "ms_per_step": round(sec * 1e3 / steps, 3),
           "schedule": {"mode": mode_name, "dw": desc["dw"], "lanes": desc["lanes"]},
           "model_bytes_per_lup": round(bpl, 4),
           "roofline": {"bound": "hbm", "kernel": "mwd_row_kernel" if mode_name == "mwd" else "naive_sweep_kernel",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "avg_launch_us": round(prof["main_ms"] * 1e3 / launches, 2)},
           "norms_fp64": desc["norms"]}
    if mode_name != "naive":
        nsec, _, ndesc, _, nstate = time_mode(S, torch, kind, dtype, (nx, ny, nz), u0_dev, co_dev, T,
                                              max(1, a.naive_steps), 1, "naive", 0, 0, R)
        del nstate
        nval = max(1, a.naive_steps) * lups / nsec / 1e9
        res["naive"] = {"value": round(nval, 3), "ms_per_step": round(nsec * 1e3 / max(1, a.naive_steps), 3),
                        "model_bytes_per_lup": ndesc["model_bytes_per_lup"]}
        res["speedup_vs_naive"] = round(value / nval, 3)
    del u0_dev, co_dev
    torch.cuda.empty_cache()
    if dtype == "f32" and not a.no_precision and "error_subrun" in w:
        res["fp32_vs_fp64"] = precision_subrun(S, torch, w, windex, n=tuple(w["error_subrun"]))
    return res


def main():
    global KERNEL_TIMING
    a = parse()
    KERNEL_TIMING = not a.no_kernel_timing
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus %d is not supported "
                                   "(the stencil path has no multi-GPU form)" % a.gpus}))
        return 2
    import torch

    import gridgen
    import paper_1410_5561_amd as S

    if a.workload == 5:
        return bench_batch(a, torch, S)
    w = workload(a.workload, a.kind)
    kind = w["kind"]
    dtype = a.dtype or (w["dtype"] if isinstance(w["dtype"], str) else w["dtype"][0])
    nx, ny, nz = w["n"]
    T = w["T"]
    R = gridgen.RADIUS[kind]
    lups = nx * ny * nz * T
    log(a, "inputs", w["name"], dtype)
    u0, co = make_inputs(w, dtype, a.workload)
    u0_dev = torch.from_numpy(u0).cuda()
    if kind in ("7c", "25c"):
        co_dev = co
    else:
        co_dev = [torch.from_numpy(c).cuda() for c in co]
    del u0
    co = None
    meter = None
    if not a.no_energy:
        from paper_1410_5561_amd import energy
        meter = energy.EnergyMeter()
    log(a, "timing MWD")
    sec, wall, desc, prof, state = time_mode(S, torch, kind, dtype, (nx, ny, nz), u0_dev, co_dev, T,
                                             a.steps, a.warmup, a.mode, a.dw, a.lanes, R, meter=meter)
    value = a.steps * lups / sec / 1e9
    main_launches = max(1, prof["main_launches"])
    model_bpl = desc["model_bytes_per_lup"]
    # roofline of the dominant kernel: algorithmic bytes (model bytes/LUP x
    # LUPs) over the time the tile kernels ran
    alg_bytes_per_launch = model_bpl * lups * a.steps / main_launches
    avg_launch_s = prof["main_ms"] / 1e3 / main_launches
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    mode_name = {0: "auto", 1: "naive", 2: "mwd"}[desc["mode"]]
    kname = "mwd_row_kernel" if mode_name == "mwd" else "naive_sweep_kernel"
    shape = "%dx%d" % (desc["dw"], desc["lanes"]) if mode_name == "mwd" else "naive"
    # measured HBM bytes per launch, from the committed rocprofv3 counter
    # summary of this kernel, workload and shape (None once the sources changed)
    from paper_1410_5561_amd import profiling
    traffic = profiling.traffic_for(kname, w["name"], dtype, shape)
    if traffic is not None:
        traffic = round(traffic)
    out = {
        "metric": "GLUP/s + rocprof bytes/LUP, MWD vs naive sweep, FP64 and FP32, 1 GPU",
        "value": round(value, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(sec * 1e3 / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w["name"], "kind": kind, "nx": nx, "ny": ny, "nz": nz, "T": T,
                   "lups_per_step": lups},
        "schedule": {"mode": mode_name, "dw": desc["dw"], "lanes": desc["lanes"],
                     "xtile": desc["xtile"], "levels": desc["levels"]},
        "step_ms": desc["step_ms"],
        "norms_fp64": desc["norms"],
        "model_bytes_per_lup": round(model_bpl, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname,
                     "algorithmic_bytes_per_launch": round(alg_bytes_per_launch),
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launches_per_step": prof["main_launches"] // a.steps,
                     "other_kernels_ms_per_step": round(prof["other_ms"] / a.steps, 4)},
    }
    if not a.no_naive and mode_name != "naive":
        log(a, "timing naive")
        nsec, _, ndesc, nprof, _ = time_mode(S, torch, kind, dtype, (nx, ny, nz), u0_dev, co_dev, T,
                                             a.naive_steps, 1, "naive", 0, 0, R, meter=meter)
        nval = a.naive_steps * lups / nsec / 1e9
        nb = ndesc["model_bytes_per_lup"]
        out["naive"] = {"value": round(nval, 3), "unit": "GLUP/s",
                        "ms_per_step": round(nsec * 1e3 / a.naive_steps, 3),
                        "model_bytes_per_lup": nb,
                        "achieved_GBs_at_model_bytes": round(nval * nb, 1)}
        out["speedup_vs_naive"] = round(value / nval, 3)
    if meter is not None:
        # energy to solution of repeated whole runs (after the timed steps),
        # from the GPU socket's energy counter
        en = {"meter": "AMD SMI energy counter of the GPU socket"}
        if not meter.ok:
            en["error"] = meter.error
        else:
            en[mode_name] = desc.get("energy")
            if not a.no_naive and mode_name != "naive":
                en["naive"] = ndesc.get("energy")
                if en[mode_name] and en["naive"]:
                    en["energy_ratio_naive_over_%s" % mode_name] = round(
                        en["naive"]["pJ_per_LUP"] / en[mode_name]["pJ_per_LUP"], 3)
        out["energy"] = en
        meter.close()
    if a.sweep:
        shapes = {1: [(4, 64), (4, 128), (4, 256), (8, 64), (8, 128), (10, 64), (16, 64)],
                  4: [(8, 64), (8, 128), (16, 64)]}[R]
        sw = []
        for dw, lx in shapes:
            try:
                ssec, _, sdesc, sprof, _ = time_mode(S, torch, kind, dtype, (nx, ny, nz), u0_dev,
                                                     co_dev, T, 2, 1, "mwd", dw, lx, R)
            except Exception as e:  # shape not compiled for this dtype
                sw.append({"dw": dw, "lanes": lx, "error": str(e)[:80]})
                continue
            sv = 2 * lups / ssec / 1e9
            sw.append({"dw": dw, "lanes": lx, "xtile": sdesc["xtile"], "GLUPs": round(sv, 2),
                       "model_bytes_per_lup": round(sdesc["model_bytes_per_lup"], 3),
                       "GBs_at_model": round(sv * sdesc["model_bytes_per_lup"], 1)})
            log(a, "sweep", sw[-1])
        out["sweep"] = sw
    if dtype == "f32" and not a.no_precision:
        log(a, "precision sub-run")
        out["fp32_vs_fp64"] = precision_subrun(S, torch, w, a.workload,
                                                n=tuple(w.get("error_subrun", (256, 256, 256))))
    if not a.no_extra and a.workload == 2:
        # the other single-grid workloads (the FP32 precision form, the
        # radius-4 star in both precisions) and the batching workload
        del state
        state = None
        del u0_dev, co_dev
        torch.cuda.empty_cache()
        extra = []
        for windex, edt in ((4, "f32"), (3, "f64"), (3, "f32")):
            extra.append(other_workload(a, torch, S, windex, edt))
        bval, bsec, bn, blups = batch_measure(a, torch, S, a.extra_steps, 1)
        extra.append({"workload": gridgen.workloads()[5]["name"], "dtype": "f32", "value": round(bval, 3),
                      "unit": "GLUP/s", "steps": a.extra_steps,
                      "ms_per_step": round(bsec * 1e3 / a.extra_steps, 3), "grids": bn})
        out["other_workloads"] = extra
        torch.cuda.empty_cache()
    if a.energy_sweep:
        if state is not None:
            del state
            state = None
        u0_dev = co_dev = None
        torch.cuda.empty_cache()
        out["energy_sweep"] = energy_sweep(a, torch, S, a.workload)
    # practical bandwidth reference: streaming copy of 2 GiB
    nbytes = 1 << 31
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    S.stencil_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        S.stencil_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9
    out["stream_copy_GBs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_stream_copy"] = round(achieved / copy_gbs, 4)
    del src, dst
    if not a.no_cpu_baseline:
        log(a, "cpu baseline")
        Tc = a.cpu_T or T
        state = None
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(w, dtype, a.workload, Tc)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
