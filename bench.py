#!/usr/bin/env python3
"""Benchmark of the ray-tracing radiative-transfer hot path on one MI355X.

Default workload: 64 SPH-like particle clouds (80% Plummer sphere + 20% logarithmic
spiral arm, Keplerian rotation, Delaunay neighbours), sizes log-uniform in
[10 000, 200 000] particles (4.1 million in all), one line sampled at 64
frequencies, the uniform HEALPix set at nside = 2 (24 antipodal pairs), FP32 sweep
with FP64 geometry.  The clouds go through the library as one batch: a disjoint
union built on the device (rt_batch) whose plan traces and solves every model in
one launch per kernel, replayed as one HIP graph.

One timed step = one replay of that graph, inputs resident in HBM: the gather of
the 64 models' chi/eta tables into the union, the walk of every ray straight into
its slot of the ray lists (slots sized by the count pass and scan that ran once
when the batch was created), the Feautrier sweep (direction by direction, each pair's
items in its own line order), the J
reduction, and the scatter of J back to the 64 models.  The cold call -- the
whole path from scratch (union build, Morton order, count pass, scan,
allocation, graph capture, one run) -- is timed once beside it.

Prints one JSON line: the metric, the rooflines of the sweep and the walk (measured
L2-miss traffic (Infinity Cache or HBM) from the committed rocprofv3 counters, and the algorithmic byte count
beside it), the other workloads' numbers, and the CPU oracle on a seeded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
F = 64

# Plan options per workload: what the autotuner (rt_autotune_plan, `--autotune`) chose on MI355X,
# kept fixed so that the timed kernel variant is the one the committed counters were taken on.
TUNED = {
    "sph_batch": dict(schedule=2, group=4, trace_lanes=4, waves_per_cu=0, n_bins=0, bins_per_octave=0),
    "wind": dict(schedule=2, group=4, trace_lanes=4, waves_per_cu=0, n_bins=0, bins_per_octave=0),
    "octree": dict(schedule=2, group=4, trace_lanes=4, waves_per_cu=0, n_bins=0, bins_per_octave=0),
    "octree_reduced": dict(schedule=2, group=4, trace_lanes=4, waves_per_cu=0, n_bins=0, bins_per_octave=0),
}


SCHEDULE_NAMES = {0: "direct launch in slot order", 1: "length-binned persistent launch",
                  2: "direct launch direction by direction over Morton-ordered origins, XCD runs of 16 (walk) and 256 (sweep) workgroups"}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_bytes(n_origins, R, total_entries, F, moving, es=4):
    """Algorithmic bytes of one sweep launch: per line point the chi and eta rows
    (2 F es), its id (4) and Z (8), its velocity (12 if moving); per pair the u row.
    Every line that passes a point counts that point's rows again (cache-served
    re-reads included)."""
    points = total_entries + n_origins * R  # every line also holds its origin
    return points * (2 * F * es + 4 + 8 + (12 if moving else 0)) + n_origins * R * F * es


def walk_bytes(n_rays, total_entries, mean_degree):
    """Algorithmic bytes of one walk launch: every step reads the current point's row of
    32-byte neighbour records (mean degree of the model), and each list entry reads one id
    and writes 12 bytes; a ray takes one step per entry plus the step that ends it."""
    return (total_entries + n_rays) * mean_degree * 32 + total_entries * 16


def src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2011_14998_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


SWEEP_SRC = ("solve.hip", "rt_internal.h")
WALK_SRC = ("trace.hip", "rt_internal.h")
KERNEL_KEYS = {"sweep": ("k_solve_direct", "k_solve_persist"), "walk": ("k_trace<1", "k_trace<2"),
               "compact": ("k_compact",), "reduce": ("k_reduce",), "gather": ("k_batch_gather",)}


def _counter_means(csv_path, counter):
    """Mean per dispatch of `counter` for each kernel family in a rocprofv3 counter CSV."""
    import csv
    acc = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            for fam, keys in list(KERNEL_KEYS.items()) + [("copy", ("copyBuffer",))]:
                if any(k in r["Kernel_Name"] for k in keys):
                    acc.setdefault(fam, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_counters(d, workload, out_json, out_md, bench_cmd):
    """Write the counter summary of one profiling session (directory d holding the rocprofv3
    outputs fetch/, write/, copyf/, copyw/, stats/ and optionally sq/, ta/) to profiles/."""
    import csv
    import glob
    f = _counter_means(glob.glob(os.path.join(d, "fetch", "*counter_collection.csv"))[0], "FETCH_SIZE")
    w = _counter_means(glob.glob(os.path.join(d, "write", "*counter_collection.csv"))[0], "WRITE_SIZE")
    cf = _counter_means(glob.glob(os.path.join(d, "copyf", "*counter_collection.csv"))[0], "FETCH_SIZE")
    cw = _counter_means(glob.glob(os.path.join(d, "copyw", "*counter_collection.csv"))[0], "WRITE_SIZE")
    # the calibration copy moves exactly 1 GiB each way per dispatch (KiB units)
    kib = 1 << 20
    fscale = kib / cf["copy"]
    wscale = kib / cw["copy"]
    res = {"workload": workload, "command": bench_cmd, "kernel_src_hash": src_hash(*SWEEP_SRC),
           "walk_src_hash": src_hash(*WALK_SRC),
           "calibration": {"copy_bytes": 1 << 30, "FETCH_SIZE_KiB": cf["copy"], "WRITE_SIZE_KiB": cw["copy"],
                           "fetch_scale": fscale, "write_scale": wscale},
           "per_launch": {}}
    for fam in ("sweep", "walk", "compact", "reduce", "gather"):
        if fam in f and fam in w:
            rb = f[fam] * 1024 * fscale
            wb = w[fam] * 1024 * wscale
            res["per_launch"][fam] = {"FETCH_SIZE_KiB": f[fam], "WRITE_SIZE_KiB": w[fam],
                                      "hbm_read_bytes": rb, "hbm_write_bytes": wb, "hbm_bytes": rb + wb}
    res["hbm_bytes_per_launch"] = res["per_launch"]["sweep"]["hbm_bytes"]
    with open(out_json, "w") as fo:
        json.dump(res, fo, indent=1)
    stats = glob.glob(os.path.join(d, "stats", "*kernel_stats.csv"))
    sq = glob.glob(os.path.join(d, "sq", "*counter_collection.csv"))
    ta = glob.glob(os.path.join(d, "ta", "*counter_collection.csv"))
    if stats and out_md:
        rows = list(csv.DictReader(open(stats[0])))
        B = bench_cmd
        with open(out_md, "w") as fo:
            fo.write(f"# Kernel times and HBM traffic: {workload}\n\n")
            fo.write("Session (run from /tmp with TMPDIR=/tmp; every command runs committed files only):\n\n")
            fo.write(f"    rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/stats -o bench -- {B}\n")
            fo.write(f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- {B}\n")
            fo.write(f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- {B}\n")
            fo.write("    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/copyf -o run -- "
                     "python3 bench.py --copy-calibration 1073741824\n")
            fo.write("    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/copyw -o run -- "
                     "python3 bench.py --copy-calibration 1073741824\n")
            if sq:
                fo.write("    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_WAVE_CYCLES "
                         f"SQ_BUSY_CYCLES SQ_WAIT_INST_ANY GRBM_GUI_ACTIVE --output-format csv -d <dir>/sq -o run -- "
                         f"{B}\n")
            if ta:
                fo.write("    rocprofv3 --pmc TA_TA_BUSY_sum TD_TD_BUSY_sum GRBM_GUI_ACTIVE --output-format csv "
                         f"-d <dir>/ta -o run -- {B}\n")
            fo.write(f"    python3 bench.py --summarize-counters <dir> {workload} {out_json} {out_md} '{B}'\n\n")
            fo.write("## rocprofv3 --stats (kernel trace)\n\n")
            fo.write("| kernel | calls | average ms | total ms | % |\n|---|---|---|---|---|\n")
            for r in rows:
                fo.write(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |\n")
            fo.write("\n## HBM traffic per launch (FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale)\n\n")
            c = res["calibration"]
            fo.write(f"Calibration: a plain 1 GiB device copy reads as FETCH_SIZE {c['FETCH_SIZE_KiB']:.0f} KiB and "
                     f"WRITE_SIZE {c['WRITE_SIZE_KiB']:.0f} KiB, so fetch_scale = {c['fetch_scale']:.4f}, "
                     f"write_scale = {c['write_scale']:.4f}.\n\n")
            fo.write("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read GB | HBM write GB | total GB |\n"
                     "|---|---|---|---|---|---|\n")
            for fam, v in res["per_launch"].items():
                fo.write(f"| {fam} | {v['FETCH_SIZE_KiB']:.0f} | {v['WRITE_SIZE_KiB']:.0f} | "
                         f"{v['hbm_read_bytes'] / 1e9:.2f} | {v['hbm_write_bytes'] / 1e9:.2f} | "
                         f"{v['hbm_bytes'] / 1e9:.2f} |\n")
            if sq:
                fo.write("\n## SQ counters per launch (sums over the device)\n\n")
                names = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_BUSY_CYCLES",
                         "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY", "GRBM_GUI_ACTIVE"]
                fo.write("| kernel | " + " | ".join(names) + " |\n|" + "---|" * (len(names) + 1) + "\n")
                for fam in ("sweep", "walk"):
                    vals = [_counter_means(sq[0], n).get(fam, float("nan")) for n in names]
                    fo.write(f"| {fam} | " + " | ".join(f"{x:.3g}" for x in vals) + " |\n")
            if ta:
                # busy fraction: the counter summed over the 256 TA/TD units over 256 x the launch's active
                # cycles per XCD (GRBM_GUI_ACTIVE summed over the 8 XCDs / 8)
                fo.write("\n## L1 data path per launch (TA/TD busy fractions)\n\n")
                fo.write("| kernel | active cycles per XCD | TA busy | TD busy | VALU instructions | "
                         "VALU issue (4-cycle estimate) |\n|---|---|---|---|---|---|\n")
                for fam in ("walk", "sweep"):
                    act = _counter_means(ta[0], "GRBM_GUI_ACTIVE").get(fam, float("nan")) / 8
                    tab = _counter_means(ta[0], "TA_TA_BUSY_sum").get(fam, float("nan")) / 256 / act
                    tdb = _counter_means(ta[0], "TD_TD_BUSY_sum").get(fam, float("nan")) / 256 / act
                    valu = _counter_means(sq[0], "SQ_INSTS_VALU").get(fam, float("nan")) if sq else float("nan")
                    fo.write(f"| {fam} | {act:.3g} | {tab:.2f} | {tdb:.2f} | {valu:.3g} | "
                             f"{valu * 4 / (1024 * act):.2f} |\n")
                fo.write("\nVALU issue: SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x active cycles), an upper estimate "
                         "for FP32 work, which can issue faster.\n")
    return res


def copy_ceiling_gbs(dev, n_bytes: int = 2 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (read + write bytes per second) of a 2 GiB
    buffer on this machine: the practical HBM ceiling beside the 8 TB/s specification."""
    import torch
    x = torch.empty(n_bytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    rate = 2.0 * n_bytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return rate


def load_traffic(workload, kernel="sweep"):
    """HBM bytes per launch of the sweep (or the walk) from the committed rocprofv3 counter
    summary of this workload, if it was taken on the kernel's current source (else None)."""
    path = os.path.join(ROOT, "profiles", f"sweep_{workload}_counters.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    if kernel == "walk":
        if d.get("walk_src_hash") != src_hash(*WALK_SRC):
            return None, path
        return d.get("per_launch", {}).get("walk", {}).get("hbm_bytes"), path
    if d.get("kernel_src_hash") != src_hash(*SWEEP_SRC):
        return None, path
    return d.get("hbm_bytes_per_launch"), path


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_threads():
    """Threads the oracle may use: the job's CPU share (OMP_NUM_THREADS where the
    environment sets it), else every core in this process's affinity set."""
    aff = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return (int(env) if env.isdigit() and int(env) > 0 else aff), aff


def cpu_baseline(parts, dirs, w2, what, budget_s=20.0):
    """The oracle (FP64, OpenMP over origins) on seeded origin samples of the same models, timed
    on this host; parts = [(model, origins)].  Its rate (solves/s) stands for the whole workload,
    which it would take the oracle far longer to finish: the record says so ("extrapolated")."""
    import oracle
    threads, aff = oracle_threads()
    solves, dt = 0, 0.0
    for m, org in parts:
        c32 = m.chi.astype(np.float32).astype(np.float64)
        e32 = m.eta.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        oracle.compute_J(m, dirs, w2, origins=org, chi=c32, eta=e32, nthreads=threads)
        dt += time.perf_counter() - t0
        solves += len(org) * len(w2) * m.F
        if dt > budget_s:
            break
    return dict(value=solves / dt, unit="point-pair-freq solves/s", cores=threads, kind="oracle",
                extrapolated=True, cpu_model=_cpu_model(), affinity_cores=aff,
                sample=f"{what}: full trace + FP64 solve + J, {solves:.3e} solves in {dt:.2f} s; the rate is "
                       f"taken for the whole workload")


def _opts_from_args(args, workload):
    o = dict(TUNED[workload])
    if args.schedule:
        o["schedule"] = {"direct": 0, "binned": 1, "spatial": 2}[args.schedule]
    if args.group:
        o["group"] = args.group
    if args.trace_lanes:
        o["trace_lanes"] = args.trace_lanes
    return o


def _timed_replays(run, steps, warmup):
    """Warm-up, then `steps` replays bracketed by HIP events on the current stream."""
    import torch
    import paper_2011_14998_amd as rt
    for _ in range(warmup):
        run()
    rt.sync_status()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        run()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rt.sync_status()
    return ev0.elapsed_time(ev1) / steps, wall / steps * 1e3


def _roofline(workload, stages, alg, dev):
    traffic, path = load_traffic(workload)
    sweep_s = stages["sweep"] * 1e-3
    r = {"kernel": "feautrier sweep", "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "achieved": None, "frac": None, "traffic": traffic, "sweep_ms": stages["sweep"],
         "measured": ("L2-to-fabric bytes per launch (the Infinity Cache or HBM serves them; an upper bound on HBM "
                      "bytes) from rocprofv3 FETCH_SIZE + WRITE_SIZE (calibrated by a "
                      "1 GiB copy) in " + os.path.relpath(path, ROOT)) if path else None}
    if traffic:
        r["achieved"] = traffic / sweep_s / 1e9
        r["frac"] = r["achieved"] / HBM_PEAK_GBS
    elif path:
        r["measured"] += " (taken on another sweep source: not used)"
    r["algorithmic"] = {"bytes_per_launch": alg, "gbs": alg / sweep_s / 1e9, "frac": alg / sweep_s / 1e9 / HBM_PEAK_GBS,
                        "model": "every line point's chi and eta rows, id, Z and velocity, counted once per line "
                                 "that reads them, plus the u rows; re-reads served by L2 and the Infinity Cache "
                                 "count too, so this fraction can exceed 1"}
    r["copy_ceiling_gbs"] = copy_ceiling_gbs(dev)
    r["note"] = ("frac is the L2-miss fraction of 8 TB/s, not the sweep's limit: the caches serve most of its table "
                 "reads (the algorithmic fraction exceeds 1) and it is held by VALU issue and the latency of L2-served loads")
    return r


def _roofline_walk(workload, stages, alg):
    traffic, path = load_traffic(workload, "walk")
    walk_s = stages["walk"] * 1e-3
    r = {"kernel": "walk", "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "achieved": None, "frac": None,
         "traffic": traffic, "walk_ms": stages["walk"],
         "measured": ("L2-to-fabric bytes per launch from the same rocprofv3 session in " + os.path.relpath(path, ROOT))
         if path else None}
    if traffic:
        r["achieved"] = traffic / walk_s / 1e9
        r["frac"] = r["achieved"] / HBM_PEAK_GBS
    elif path:
        r["measured"] += " (taken on another walk source: not used)"
    r["algorithmic"] = {"bytes_per_launch": alg, "gbs": alg / walk_s / 1e9, "frac": alg / walk_s / 1e9 / HBM_PEAK_GBS,
                        "model": "per step the current point's row of 32-byte neighbour records at the model's mean "
                                 "degree, per list entry a 4-byte id read and 12 bytes written; re-reads served by "
                                 "the caches count too"}
    return r


def _other_wind(rt, torch, dev, steps=10):
    """The 50 000-point analytic wind at nside 4 (one plan), as an extra line of numbers."""
    import synth
    m = synth.wind_model(seed=2, P=50_000, F=F)
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(4)
    chi, eta = torch.as_tensor(c32, device=dev), torch.as_tensor(e32, device=dev)
    I_bc = torch.as_tensor(m.I_bc, dtype=torch.float64, device=dev)
    J = torch.empty((m.P, F), dtype=torch.float32, device=dev)
    plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, n_origins=m.P, precision=rt.RT_F32,
                   **TUNED["wind"])
    ms, _ = _timed_replays(lambda: plan.run(use_graph=True), steps, 2)
    st = plan.profile(3)
    total = plan.info()["total"]
    out = {"workload": "analytic spherical wind, 50000 points, nside 4 (96 pairs), F=64, FP32 sweep",
           "solves_per_s": m.P * ds.R * F / (ms * 1e-3), "ms_per_step": ms, "stages_ms": st,
           "sweep_algorithmic_frac": sweep_bytes(m.P, ds.R, total, F, True) / (st["sweep"] * 1e-3) / 1e9 /
           HBM_PEAK_GBS}
    del plan
    rt.release_cached_memory()
    return out


def run_batch(args, rt, torch, dev):
    """The default workload: 64 SPH-like clouds through rt_batch."""
    import synth
    t_gen = time.perf_counter()
    gen_workers = min(16, oracle_threads()[0])
    ms_ = synth.sph_batch_models(n_models=64, scale=args.batch_scale, workers=gen_workers)
    P_tot = sum(m.P for m in ms_)
    _log(f"generated 64 SPH-like clouds: {P_tot} particles, {sum(m.E for m in ms_)} neighbour entries in "
         f"{time.perf_counter() - t_gen:.1f} s")
    models, chis, etas, Js = [], [], [], []
    for m in ms_:
        c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
        models.append(rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel))
        chis.append(torch.as_tensor(c32, device=dev))
        etas.append(torch.as_tensor(e32, device=dev))
        Js.append(torch.empty((m.P, F), dtype=torch.float32, device=dev))
    nside = args.nside or 2
    ds = rt.DirSet.uniform(nside)
    R = ds.R
    I_bc = torch.as_tensor(ms_[0].I_bc, dtype=torch.float64, device=dev)
    opts = _opts_from_args(args, "sph_batch")
    _log(f"building the batch (union on the device, count pass, graph) with {opts} ...")
    t0 = time.perf_counter()
    b = rt.Batch(models, ds, chis, etas, ms_[0].freq.len, ms_[0].freq.dx, I_bc, Js, precision=rt.RT_F32, **opts)
    torch.cuda.synchronize()
    _log(f"batch built in {time.perf_counter() - t0:.1f} s")
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        opts, tms = b.autotune(n_runs=2, verbose=True)
        tuned = dict(opts, ms_per_step=tms, seconds=time.perf_counter() - t0)
        _log(f"autotuner chose {opts}")
    total = b.info()["total"]
    ms, wall_ms = _timed_replays(lambda: b.run(use_graph=True), args.steps, args.warmup)
    _log(f"step {ms:.3f} ms ({wall_ms:.3f} ms wall)")
    stages = b.profile(max(3, min(args.steps, 5)))
    _log("stages (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
    solves = P_tot * R * F
    alg = sweep_bytes(P_tot, R, total, F, moving=True)
    roof = _roofline("sph_batch", stages, alg, dev)
    desc = (f"64 SPH-like clouds (80% Plummer sphere + 20% logarithmic spiral arm, Keplerian rotation, Delaunay "
            f"neighbours), sizes log-uniform in [10000, 200000] x {args.batch_scale}, {P_tot} particles in all; "
            f"nside {nside} ({R} pairs), F={F}, FP32 sweep, FP64 tracing; one disjoint union built on the device, "
            "one HIP graph")
    rec = {
        "metric": "point-ray-freq solves/s (one solve = one origin x antipodal ray pair x frequency)",
        "value": solves / (ms * 1e-3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 sweep, f64 geometry", "data": "synthetic (seeded SPH-like clouds)",
        "config": {"workload": desc, "models": 64, "points": P_tot, "pairs_per_point": R, "freqs": F,
                   "ray_list_entries": total, "mean_line_length": (total + P_tot * R) / (P_tot * R),
                   "plan_options": opts, "autotune": tuned,
                   "timed_step": "one replay of the batch's HIP graph: table gather into the union, walk of every "
                                 "ray into its slot (slots from the count pass and scan at creation, rays in "
                                 "windows of 64 origins ordered by length), sweep ("
                                 + SCHEDULE_NAMES[opts["schedule"]] + "), J reduction, J scatter to the 64 models"},
        "roofline": roof,
        "roofline_walk": _roofline_walk("sph_batch", stages,
                                        walk_bytes(P_tot * 2 * R, total, sum(m.E for m in ms_) / P_tot)),
        "stages_ms": stages,
        "line_point_freq_updates_per_s": (total + P_tot * R) * F / (ms * 1e-3),
    }
    del b
    rt.release_cached_memory()
    torch.cuda.empty_cache()
    if not args.no_cold:
        _log("cold call: rt_compute_J_batched from scratch ...")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt.compute_J_batched(models, ds, chis, etas, ms_[0].freq.len, ms_[0].freq.dx, I_bc, Js=Js, **opts)
        torch.cuda.synchronize()
        cold = time.perf_counter() - t0
        rt.release_cached_memory()
        rec["cold_call"] = {"s": cold, "what": "rt_compute_J_batched from scratch: union built on the device, "
                                               "Morton order of every model, count pass, scan, length order, "
                                               "allocation of the lists, graph capture, one run, destruction"}
    return rec, ms_, ds


def run_plan_workload(args, rt, torch, dev):
    """One model through one plan: the wind (50k points, nside 4) or the AMR-octree-like clouds."""
    import synth
    t_gen = time.perf_counter()
    if args.workload == "wind":
        m = synth.wind_model(seed=2, P=50_000, F=F)
        nside = args.nside or 4
        desc = "analytic spherical wind, 50000 points (Delaunay), moving (v_inf 20 Doppler widths)"
    else:
        target = 500_000 if args.workload == "octree" else 50_000
        m = synth.octree_model(seed=3, target=target)
        nside = args.nside or 4
        desc = (f"AMR-octree-like cloud, {m.P} leaves (levels 5-8, touching-leaf neighbours), 2 lines x 48 "
                "frequencies, turbulent velocity 3 Doppler widths rms")
    _log(f"generated {args.workload}: {m.P} points, {m.E} neighbour entries in {time.perf_counter() - t_gen:.1f} s")
    Fw = m.F
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(nside)
    R = ds.R
    chi, eta = torch.as_tensor(c32, device=dev), torch.as_tensor(e32, device=dev)
    I_bc = torch.as_tensor(m.I_bc, dtype=torch.float64, device=dev)
    J = torch.empty((m.P, Fw), dtype=torch.float32, device=dev)
    scheme = {"feautrier2": rt.SCHEME_FEAUTRIER2, "hermite": rt.SCHEME_HERMITE}[args.scheme]
    opts = _opts_from_args(args, args.workload)
    plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, n_origins=m.P, precision=rt.RT_F32,
                   dtau_max=args.dtau_max, dv_max=args.dv_max, scheme=scheme,
                   walk={"exact": rt.WALK_EXACT, "padded": rt.WALK_PADDED, "two-pass": rt.WALK_TWO_PASS}[args.walk],
                   **opts)
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        opts, tms = rt.autotune(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, n_origins=m.P, n_runs=2,
                                verbose=True, dtau_max=args.dtau_max, dv_max=args.dv_max, scheme=scheme)
        tuned = dict(opts, ms_per_step=tms, seconds=time.perf_counter() - t0)
        plan.retune(**opts)
    total = plan.info()["total"]
    ms, wall_ms = _timed_replays(lambda: plan.run(use_graph=True), args.steps, args.warmup)
    _log(f"step {ms:.3f} ms ({wall_ms:.3f} ms wall)")
    stages = plan.profile(max(3, min(args.steps, 10)))
    _log("stages (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
    alg = sweep_bytes(m.P, R, total, Fw, moving=m.vel is not None)
    rec = {
        "metric": "point-ray-freq solves/s (one solve = one origin x antipodal ray pair x frequency)",
        "value": m.P * R * Fw / (ms * 1e-3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 sweep, f64 geometry", "data": f"synthetic (seeded {args.workload})",
        "config": {"workload": f"{desc}; nside {nside} ({R} pairs), F={Fw}, FP32 sweep", "points": m.P,
                   "pairs_per_point": R, "freqs": Fw, "ray_list_entries": total,
                   "mean_line_length": (total + m.P * R) / (m.P * R), "plan_options": opts, "walk": args.walk,
                   "dtau_max": args.dtau_max, "dv_max": args.dv_max, "scheme": args.scheme, "autotune": tuned,
                   "frequency_chunks_per_pair": (Fw + 63) // 64,
                   "timed_step": "one replay of the plan's HIP graph: walk of every ray into its slot (slots from "
                                 "the count pass and scan at creation, rays in windows of 64 origins ordered by "
                                 "length), sweep (" + SCHEDULE_NAMES[opts["schedule"]]
                                 + "), J reduction"},
        "roofline": _roofline(args.workload if nside == 4 else args.workload + f"_nside{nside}", stages, alg, dev),
        "roofline_walk": _roofline_walk(args.workload if nside == 4 else args.workload + f"_nside{nside}", stages,
                                        walk_bytes(m.P * 2 * R, total, m.E / m.P)),
        "stages_ms": stages,
        "line_point_freq_updates_per_s": (total + m.P * R) * Fw / (ms * 1e-3),
    }
    del plan
    rt.release_cached_memory()
    return rec, [m], ds


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["sph_batch", "wind", "octree", "octree_reduced", "closure", "precision",
                                           "directions", "mlp"],
                    default="sph_batch",
                    help="sph_batch: 64 SPH-like clouds in one batch (default, --batch-scale 1: 4.1M particles); "
                         "wind: the 50k-point wind at nside 4; octree: ~500k-leaf AMR-like cloud, 2x48 "
                         "frequencies; octree_reduced: the same field with ~50k leaves; closure: the learned "
                         "closure trained on winds of seeds 500-503 and tested on 510-511 against the plain "
                         "nside-8 solve (--closure-points each); precision: the FP32 sweep's error against the "
                         "FP64 oracle, model by model; directions: adaptive (l 1..4) against regular nside-16 "
                         "directions on the AMR-like cloud")
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner on this workload first (otherwise the fixed options in TUNED)")
    ap.add_argument("--schedule", choices=["direct", "binned", "spatial"], default=None)
    ap.add_argument("--group", type=int, default=0, help="sweep load-group size (4 or 8)")
    ap.add_argument("--trace-lanes", type=int, default=0, help="lanes per ray in the walk (4, 8 or 16)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="origins per model timed on the CPU oracle (0 = skip; -1 = the workload's default)")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold-call timing")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra workloads' numbers")
    ap.add_argument("--nside", type=int, default=0, help="HEALPix nside (0 = the workload's own)")
    ap.add_argument("--summarize-counters", nargs=5, metavar=("DIR", "WORKLOAD", "OUT_JSON", "OUT_MD", "CMD"),
                    help="summarise a rocprofv3 session directory into the profiles/ files and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (for scaling HBM counters) and exit")
    ap.add_argument("--walk", choices=["exact", "padded", "two-pass"], default="exact",
                    help="plan walk: once into the creation-time slots (default), once into padded slots plus "
                         "compaction, or count + write")
    ap.add_argument("--closure-points", type=int, default=2_000_000, help="points per closure model")
    ap.add_argument("--closure-family", choices=["wind", "octree"], default="wind",
                    help="closure models: analytic winds, or AMR-octree-like clouds (about --closure-points leaves)")
    ap.add_argument("--closure-train", type=int, default=4, help="closure training models (seeds 500..)")
    ap.add_argument("--closure-test", type=int, default=2, help="closure test models (seeds 510..)")
    ap.add_argument("--closure-steps", type=int, default=20000, help="closure training steps")
    ap.add_argument("--closure-batch", type=int, default=8192)
    ap.add_argument("--closure-coarse-nside", type=int, default=1,
                    help="nside of the coarse solve the closure corrects (1: 6 pairs, 2: 24, 4: 96)")
    ap.add_argument("--closure-lr", type=float, default=2e-3)
    ap.add_argument("--mlp-train-steps", type=int, default=1000,
                    help="mlp workload: graph-replayed training steps per timed call")
    ap.add_argument("--dv-max", type=float, default=0.0,
                    help="adaptive velocity sampling: split line intervals whose projected velocity changes by "
                         "more than this many Doppler widths (0 = off)")
    ap.add_argument("--dtau-max", type=float, default=0.0,
                    help="adaptive optical-depth increments: split line intervals to at most this optical depth "
                         "(0 = off)")
    ap.add_argument("--scheme", choices=["feautrier2", "hermite"], default="feautrier2",
                    help="rows of the line solve: second-order Feautrier, or the fourth-order Hermitian rows "
                         "(steps must stay below about 3.46: use --dtau-max)")
    args = ap.parse_args()
    if args.summarize_counters:
        d, wl, oj, om, cmd = args.summarize_counters
        print(json.dumps(summarize_counters(d, wl, oj, om, cmd), indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of "
                                   "this build (the path shards by origins, see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2011_14998_amd as rt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return
    rt.load()
    if args.workload == "closure":
        run_closure(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "directions":
        run_directions(args)
        return
    if args.workload == "mlp":
        run_mlp(args)
        return
    if args.workload == "sph_batch":
        rec, models, ds = run_batch(args, rt, torch, dev)
        per_model = 600 if args.cpu_sample < 0 else args.cpu_sample
    else:
        rec, models, ds = run_plan_workload(args, rt, torch, dev)
        per_model = (25_000 if args.workload == "wind" else 3000) if args.cpu_sample < 0 else args.cpu_sample
    if not args.no_extra and args.workload == "sph_batch":
        _log("extra numbers: the 50k wind at nside 4 ...")
        rec["other_workloads"] = {"wind50k_nside4": _other_wind(rt, torch, dev)}
    if per_model > 0:
        from oracle import dirset_uniform
        _, dirs, w2 = dirset_uniform(int(round(np.sqrt(ds.R / 6))))
        rng = np.random.default_rng(7)
        parts = [(m, np.sort(rng.choice(m.P, min(per_model, m.P), replace=False)).astype(np.int32))
                 for m in models]
        what = (f"{per_model} seeded origins of each of the {len(models)} models" if len(models) > 1
                else f"{per_model} seeded origins of the model")
        _log(f"timing the CPU oracle ({what}) ...")
        rec["cpu_baseline"] = cpu_baseline(parts, dirs, w2, what)
    print(json.dumps(rec), flush=True)


# multiply-adds per sample of the closure network (16 -> 256 -> 256 -> 256 -> 2), as FLOPs
MLP_FWD_FLOP = 2 * (16 * 256 + 2 * 256 * 256 + 256 * 2)
# backward: the two hidden products of the signal pass (dZ W^T for W3, W2) and the weight
# gradients of W1..W3 (H^T dZ); the head and elementwise work are not counted
MLP_BWD_FLOP = 2 * (2 * 256 * 256) + 2 * (16 * 256 + 2 * 256 * 256)


def run_mlp(args):
    """The closure network alone: inference over 6.4M samples (100 000 points x 64 frequencies),
    the backward at the training batch, and whole training steps replayed from one captured
    graph (rt_mlp_train); HIP-event times, FLOPs of the matrix products, one JSON line."""
    import torch

    import paper_2011_14998_amd as rt

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    N, n_inf, batch = 1_000_000, 6_400_000, args.closure_batch
    X = torch.randn((N, 16), generator=g, device=dev).to(torch.bfloat16).view(torch.int16)
    T = torch.randn(N, generator=g, device=dev)
    rows_inf = torch.randint(0, N, (n_inf,), generator=g, device=dev, dtype=torch.int32)
    net = rt.MLP(seed=1)
    Y = torch.empty((n_inf, 2), dtype=torch.float32, device=dev)

    def timed(fn, reps, warm_s=0.5):
        # untimed warm-up of at least warm_s seconds, so that the clocks have settled
        t0 = time.perf_counter()
        while True:
            fn()
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= warm_s:
                break
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(args.steps, 5)
    t_inf = timed(lambda: net.forward(X, rows=rows_inf, Y=Y), reps)
    rows = torch.randint(0, N, (batch,), generator=g, device=dev, dtype=torch.int32)
    Yb = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    net.forward(X, rows=rows, Y=Yb, keep=True)
    dY = rt.mlp_nll(Yb, T, rows=rows)
    t_fwd_keep = timed(lambda: net.forward(X, rows=rows, Y=Yb, keep=True), reps)
    net.forward(X, rows=rows, Y=Yb, keep=True)
    t_bwd = timed(lambda: net.backward(X, dY, rows=rows), reps)
    # the backward at a batch large enough that the per-kernel floor no longer dominates
    big = 65536
    rows_big = torch.randint(0, N, (big,), generator=g, device=dev, dtype=torch.int32)
    Ybig = torch.empty((big, 2), dtype=torch.float32, device=dev)
    dYbig = rt.mlp_nll(net.forward(X, rows=rows_big, Y=Ybig, keep=True), T, rows=rows_big)
    net.forward(X, rows=rows_big, Y=Ybig, keep=True)
    t_bwd_big = timed(lambda: net.backward(X, dYbig, rows=rows_big), reps)
    steps = args.mlp_train_steps
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    kw = dict(batch=batch, total_steps=steps * 10, lr=1e-3, lr_final=1e-5, loss_sum=loss)
    t_step = timed(lambda: net.train(X, T, steps, **kw), 2, warm_s=0.0) / steps
    rec = {
        "metric": "closure network: inference and training rates on the matrix cores",
        "value": MLP_FWD_FLOP * n_inf / (t_inf * 1e-3) / 1e12,
        "unit": "TFLOP/s (inference, BF16 MFMA, FP32 accumulate)",
        "n_gpus": 1, "steps": reps, "warmup": "0.5 s of untimed calls", "ms_per_step": t_inf, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic (random inputs and weights)",
        "config": {"workload": f"MLP 16-256-256-256-2, inference over {n_inf} samples, training batch {batch}"},
        "inference": {"samples": n_inf, "ms": t_inf, "tflops": MLP_FWD_FLOP * n_inf / (t_inf * 1e-3) / 1e12,
                      "frac_of_2.5PF": MLP_FWD_FLOP * n_inf / (t_inf * 1e-3) / 2.5e15},
        "forward_keep": {"samples": batch, "ms": t_fwd_keep,
                         "tflops": MLP_FWD_FLOP * batch / (t_fwd_keep * 1e-3) / 1e12},
        "backward": {"samples": batch, "ms": t_bwd, "tflops": MLP_BWD_FLOP * batch / (t_bwd * 1e-3) / 1e12,
                     "frac_of_2.5PF": MLP_BWD_FLOP * batch / (t_bwd * 1e-3) / 2.5e15},
        "backward_65536": {"samples": big, "ms": t_bwd_big,
                           "tflops": MLP_BWD_FLOP * big / (t_bwd_big * 1e-3) / 1e12,
                           "frac_of_2.5PF": MLP_BWD_FLOP * big / (t_bwd_big * 1e-3) / 2.5e15},
        "train_step_graph": {"samples": batch, "ms": t_step, "steps_timed": 2 * steps,
                             "tflops": (MLP_FWD_FLOP + MLP_BWD_FLOP) * batch / (t_step * 1e-3) / 1e12},
    }
    print(json.dumps(rec), flush=True)


def run_precision(args):
    """FP32 sweep (FP64 geometry) and FP64 sweep against the FP64
    oracle fed the same FP32 table values, on seeded origin samples of each model; one JSON line."""
    import torch

    import oracle
    import paper_2011_14998_amd as rt
    import synth

    threads = min(len(os.sched_getaffinity(0)), 16)
    cases = [
        ("homogeneous sphere, 1200 points, nside 1, F=31", lambda: synth.sphere_model(), 1, None),
        ("analytic wind, 50000 points, nside 4, F=64", lambda: synth.wind_model(seed=2, P=50_000), 4, 1500),
        ("AMR-octree-like cloud, ~50000 leaves, nside 4, 2x48 freqs",
         lambda: synth.octree_model(seed=3, target=50_000), 4, 400),
        ("SPH-like cloud (Plummer + spiral arm), 20000 particles, nside 2, F=64",
         lambda: synth.sph_cloud_model(seed=400, P=20_000), 2, 1500),
    ]
    out = []
    for name, make, nside, n_sample in cases:
        m = make()
        rng = np.random.default_rng(11)
        org = (np.arange(m.P) if n_sample is None or n_sample >= m.P
               else np.sort(rng.choice(m.P, n_sample, replace=False))).astype(np.int32)
        c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
        _, dirs, w2 = oracle.dirset_uniform(nside)
        t0 = time.perf_counter()
        Jo = oracle.compute_J(m, dirs, w2, origins=org, chi=c64, eta=e64, nthreads=threads)
        t_or = time.perf_counter() - t0
        model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
        ds = rt.DirSet.uniform(nside)
        o_t = torch.as_tensor(org, device="cuda")
        I_bc = torch.as_tensor(m.I_bc, dtype=torch.float64, device="cuda")
        rec = dict(model=name, points=m.P, origins=len(org), freqs=m.F, pairs=ds.R, oracle_s=t_or)
        for prec, tab, dt in ((rt.RT_F32, (c32, e32), torch.float32), (rt.RT_F64, (c64, e64), torch.float64)):
            chi = torch.as_tensor(tab[0], device="cuda")
            eta = torch.as_tensor(tab[1], device="cuda")
            J = torch.empty((len(org), m.F), dtype=dt, device="cuda")
            plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, origins=o_t, precision=prec,
                           schedule=rt.SCHED_SPATIAL)
            plan.run()
            rt.sync_status()
            e = np.abs(J.double().cpu().numpy() - Jo) / np.abs(Jo)
            key = "fp32" if prec == rt.RT_F32 else "fp64"
            rec[key] = dict(max_rel=float(e.max()), median_rel=float(np.median(e)),
                            p99_rel=float(np.quantile(e, 0.99)))
            del plan
        _log(f"{name}: fp32 max {rec['fp32']['max_rel']:.2e}, fp64 max {rec['fp64']['max_rel']:.2e}")
        out.append(rec)
    print(json.dumps({"metric": "relative error of J against the FP64 oracle, per model", "per_model": out}),
          flush=True)


def run_directions(args, n_origins=1000, n_sample=10_000):
    """Section 3.2.1's comparison on the AMR-like cloud (~50 000 leaves): the adaptive
    set l = 1..4 (276 pairs, 552 rays, refined towards the point density seen from each
    origin) against the regular nside-16 set (1536 pairs, 3072 rays).  Per pair: the
    adaptive leaf containing a regular pair's direction is compared with that pair's u;
    per point: J.  Times are plan replays of the whole path.  One JSON line."""
    import torch

    import paper_2011_14998_amd as rt
    import synth

    m = synth.octree_model(seed=3, target=50_000)
    _log(f"AMR-like cloud: {m.P} leaves, F = {m.F}")
    rng = np.random.default_rng(21)
    org_h = np.sort(rng.choice(m.P, min(n_origins, m.P), replace=False)).astype(np.int32)
    sample = rng.choice(m.P, min(n_sample, m.P), replace=False).astype(np.int32)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    chi, eta = torch.as_tensor(c32, device="cuda"), torch.as_tensor(e32, device="cuda")
    I_bc = torch.as_tensor(m.I_bc, dtype=torch.float64, device="cuda")
    org = torch.as_tensor(org_h, device="cuda")
    n_o = len(org_h)
    reg = rt.DirSet.uniform(16)
    ada = rt.DirSet.adaptive(model, 1, 4, torch.as_tensor(sample, device="cuda"), origins=org)
    out = {}
    for name, ds in (("regular", reg), ("adaptive", ada)):
        J = torch.empty((n_o, m.F), dtype=torch.float32, device="cuda")
        plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, origins=org, precision=rt.RT_F32,
                       schedule=rt.SCHED_SPATIAL)
        plan.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            plan.run()
        e1.record()
        e1.synchronize()
        out[name] = dict(J=J.double().cpu().numpy(), u=plan.copy_u().double().cpu().numpy(),
                         ms=e0.elapsed_time(e1) / 3, pairs=ds.R)
        rt.sync_status()
        _log(f"{name}: {ds.R} pairs, {out[name]['ms']:.2f} ms per run")
        del plan
    # regular pair -> adaptive leaf, per origin
    _, _, rdirs, _ = reg.export()
    apix, alev, _, _ = ada.export()
    lut_pix = {}
    for lv in range(1, 5):
        ns = 1 << lv
        p = rt.healpix_vec2pix(ns, rdirs)
        q = rt.healpix_vec2pix(ns, -rdirs)
        lut_pix[lv] = (np.minimum(p, q), 12 * ns * ns)
    u_reg, u_ada = out["regular"]["u"], out["adaptive"]["u"]
    errs = []
    for o in range(n_o):
        leaf = np.full(len(rdirs), -1, np.int64)
        for lv in range(1, 5):
            canon, npix = lut_pix[lv]
            lut = np.full(npix, -1, np.int64)
            sel = alev[o] == lv
            lut[apix[o][sel]] = np.nonzero(sel)[0]
            hit = lut[canon]
            leaf = np.where((leaf < 0) & (hit >= 0), hit, leaf)
        assert np.all(leaf >= 0)
        errs.append(np.abs(u_ada[o][leaf] - u_reg[o]) / np.abs(u_reg[o]))
    e = np.concatenate([x.ravel() for x in errs])
    eJ = np.abs(out["adaptive"]["J"] - out["regular"]["J"]) / np.abs(out["regular"]["J"])
    rec = {
        "metric": "adaptive (l 1..4, 552 rays) vs regular (nside 16, 3072 rays) directions: ray-pair and J relative "
                  "errors, speedup of the whole path",
        "value": out["regular"]["ms"] / out["adaptive"]["ms"], "unit": "x (regular time / adaptive time)",
        "n_gpus": 1, "higher_is_better": True,
        "config": {"workload": f"AMR-like cloud, {m.P} leaves, 2x48 frequencies, {n_o} seeded origins, sample of "
                               f"{len(sample)} points for the refinement", "origins": n_o},
        "pairs": {"regular": out["regular"]["pairs"], "adaptive": out["adaptive"]["pairs"]},
        "ms": {"regular": out["regular"]["ms"], "adaptive": out["adaptive"]["ms"]},
        "pair_error_cdf": {str(t): float(np.mean(e < t)) for t in (1e-3, 1e-2, 0.1, 0.2)},
        "J_error": {"median": float(np.median(eJ)), "p90": float(np.quantile(eJ, 0.9)), "max": float(eJ.max())},
    }
    print(json.dumps(rec), flush=True)


def _gen_model(spec):
    """One closure model: an analytic wind of P points, or an AMR-octree-like cloud of about P leaves."""
    import synth
    family, seed, P = spec
    _log(f"generating {family} seed {seed} ({P} points) ...")
    t0 = time.perf_counter()
    m = synth.wind_model(seed=seed, P=P) if family == "wind" else synth.octree_model(seed=seed, target=P)
    return m, time.perf_counter() - t0


def _mem_line(torch, rt) -> str:
    free, total = torch.cuda.mem_get_info()
    return (f"device memory in use {(total - free) / 2**30:.1f} GiB (torch reserved "
            f"{torch.cuda.memory_reserved() / 2**30:.1f} GiB, plan cache {rt.cached_memory() / 2**30:.1f} GiB, "
            f"live plans {rt.plan_memory() / 2**30:.1f} GiB)")


def run_closure(args):
    """Learned closure vs the plain nside-8 solve: label, train, test; one JSON line."""
    import math
    from concurrent.futures import ProcessPoolExecutor, as_completed

    import torch

    import paper_2011_14998_amd as rt
    from paper_2011_14998_amd import closure as cl

    P = args.closure_points
    fam = args.closure_family
    seeds_train = [500 + i for i in range(args.closure_train)]
    seeds_test = [510 + i for i in range(args.closure_test)]
    models = {}
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(8, len(seeds_train) + len(seeds_test))) as ex:
        futs = [ex.submit(_gen_model, (fam, s, P)) for s in seeds_train + seeds_test]
        for f in as_completed(futs):
            m, sec = f.result()
            models[m.meta["seed"]] = m
            _log(f"generated {fam} seed {m.meta['seed']}: {m.P} points, {m.E} entries ({sec:.0f} s)")
    gen_s = time.perf_counter() - t0
    nc = args.closure_coarse_nside
    ds1, ds2, ds8 = rt.DirSet.uniform(nc), rt.DirSet.uniform(2), rt.DirSet.uniform(8)
    labs = []
    t0 = time.perf_counter()
    for sd in seeds_train:
        dm = cl.DeviceModel.from_synth(models.pop(sd))
        labs.append(cl.label(dm, ds1, ds8, verbose=True))
        _log(f"labelled seed {sd}: nside-{nc} {labs[-1].coarse.ms:.0f} ms, nside-8 {labs[-1].fine.ms:.0f} ms; "
             + _mem_line(torch, rt))
    label_s = time.perf_counter() - t0
    X, T, norm = cl.dataset(labs)
    del labs
    _log(f"training set: {X.shape[0]} samples")
    t0 = time.perf_counter()
    net = cl.train(X, T, norm, steps=args.closure_steps, batch=args.closure_batch, lr=args.closure_lr, seed=7,
                   log_every=max(1, args.closure_steps // 10))
    train_s = time.perf_counter() - t0
    del X, T
    torch.cuda.empty_cache()
    fractions = [0.0, 0.1, 0.25, 0.5, 1.0]
    results = []
    for sd in seeds_test:
        dm = cl.DeviceModel.from_synth(models.pop(sd))
        lab = cl.label(dm, ds1, ds8, verbose=True)
        # warm timing of both paths: the labelling runs above include first-launch costs
        r = cl.evaluate(net, lab, ds1, ds8, fractions, mid_set=ds2, verbose=True)
        results.append(r)
        del lab, dm
        torch.cuda.empty_cache()
    # headline: per target fallback fraction, error and time over the test models
    curves = [r.get("fallback_for_target") for r in results]
    summary = []
    for i, q in enumerate(fractions):
        runs = [r["closure"][i] for r in results]
        plain = sum(r["plain_ms"] for r in results)
        tot = sum(c["total_ms"] for c in runs)
        summary.append(dict(target_fraction=q, median=float(np.median([c["median"] for c in runs])),
                            median_unflagged=float(np.median([c["median_unflagged"] for c in runs])),
                            p99=float(np.median([c["p99"] for c in runs])),
                            flagged_fraction=float(np.mean([c["flagged_fraction"] for c in runs])),
                            closure_ms=tot, plain_ms=plain, speedup=plain / tot))
    ok = [s for s in summary if s["median"] <= 1e-3 and s["target_fraction"] < 1.0]
    head = max(ok, key=lambda s: s["speedup"]) if ok else summary[0]
    rec = {
        "metric": "learned closure vs plain nside-8 solve: speedup at the smallest fallback fraction with median "
                  "J rel err <= 1e-3 (if none reaches it: without fallback, with its error)",
        "value": head["speedup"],
        "unit": "x (plain time / closure time)",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": head["closure_ms"] / len(results),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 mfma / f32 accumulate (network), f32 sweep, f64 geometry",
        "data": "synthetic (seeded analytic winds)" if fam == "wind" else "synthetic (seeded AMR-octree-like clouds)",
        "config": {"workload": f"learned closure, {fam} models of {P} points, train seeds {seeds_train}, test "
                               f"seeds {seeds_test}; coarse nside {nc}, fine nside 8, F={results[0]['F']}",
                   "family": fam,
                   "points": P, "train_models": len(seeds_train), "test_models": len(seeds_test),
                   "steps": args.closure_steps, "batch": args.closure_batch, "lr": args.closure_lr},
        "headline": head, "fallback_sweep": summary, "per_model": results,
        "fallback_needed_for_1e-3": curves,
        "training": {"loss_history": net.history, "train_s": train_s, "label_s": label_s, "generate_s": gen_s},
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
