#!/usr/bin/env python3
"""Throughput of the layer-case FDM transport hot path on one MI355X.

Workload: the single-instance configuration at scale -- a 2048 x 2048
periodic grid holding a circular dislocation loop (radius 300 cells,
Gaussian cross-section sigma = 6, amplitude 1), LAW Hamiltonian with uniform
celerity v0 = -1 (expansion), superbee limiter, two-stage Heun steps at
Courant number 0.4 (synthetic input, float32 state).

A step is one full time step of every node (both stages: limited slopes,
one-sided derivatives, speeds, numerical Hamiltonian, conservative update),
replayed from a captured HIP graph, plus the per-chunk FP64 diagnostics.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
BYTES_PER_CELL_STEP = 16        # read + write alpha_11 and alpha_12 once (float32; 32 for float64)
# One VALU lane-operation per lane per cycle (packed FP32 is not used):
# 256 CUs x 64 lanes x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# FP32 operations of one node-stage counted from the scheme's definition:
# two limited slopes (12 each), four one-sided derivatives (8), four corner
# Hamiltonians with gradients (32), four speeds (16), weights (12), the
# weighted sum and viscosity terms (19), update and stage combination (9).
OPS_PER_NODE_STAGE = 120
# VALU instructions the compiled node function (LAW, superbee) issues per
# node-stage: SQ_INSTS_VALU per wave over the node-stages the wave computes,
# 85 for the fused kernel's loop and the stage kernel alike.  Fewer than the
# operations of the definition: FMA, med3 and three-operand max/min each do
# two or three of them in one issue.
ISSUED_PER_NODE_STAGE = 85


# Per-launch memory traffic of the stage kernel, measured with rocprofv3
# counters (FETCH_SIZE and WRITE_SIZE passes, each calibrated by a plain copy
# kernel of known size) and tied to the kernel sources it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_loop_2048_fp32_traffic.json")
KERNEL_SOURCES = ["fdm_stage.h", "fdm_stage_f32.hip", "fdm_internal.h", "fdm_kernels.hip"]
STAGE_NAMES = {"fwd": "stage_kernel<float, float, 2, 0, false, 0, false>",
               "heun2": "stage_kernel<float, float, 2, 0, false, 2, false>",
               "fused": "fused_kernel<2, 0, false, false>"}
COPY_NAME = "copy_kernel<float>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1911_03225_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _counter_means(directories, counter):
    """Mean counter value (KiB per dispatch) per kernel family over rocprofv3
    CSV directories (comma-separated); families absent from them are left out."""
    import csv
    import glob
    files = [f for d in directories.split(",") for f in glob.glob(os.path.join(d, "*counter_collection.csv"))]
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % directories)
    import collections
    # (family, grid size) -> values; the copy probe's own stage launch has the
    # same kernel name on a larger grid, so each family keeps its most
    # frequent grid size (the bench launches)
    vals = collections.defaultdict(list)
    grids = collections.defaultdict(list)
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            fam = [k for k, pat in STAGE_NAMES.items() if pat in name]
            if COPY_NAME in name:
                fam = ["copy"]
            if fam:
                vals[(fam[0], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    out, grid = {}, {}
    for k in list(STAGE_NAMES) + ["copy"]:
        groups = [(len(v), g, v) for (fam, g), v in vals.items() if fam == k]
        if not groups:
            if k == "copy":
                raise SystemExit("no %s samples for the copy probe in %s" % (counter, directories))
            continue
        _, grid[k], v = max(groups)
        out[k] = sum(v) / len(v)
    by_grid = {(fam, g): sum(v) / len(v) for (fam, g), v in vals.items()}
    return out, grid, by_grid


def rows_from_grid(grid_threads, n, strip=60):
    """Tile height of a stage launch on an n x n grid from its thread count:
    blocks of 4 waves, rounded up to a multiple of 8 blocks (one per XCD);
    strip: output columns per wave (56 for the fused kernel)."""
    strips = -(-n // strip)
    for r in range(1, n + 1):
        tiles = strips * -(-n // r)
        blocks = -(-tiles // 4)
        blocks = -(-blocks // 8) * 8
        if blocks * 256 == grid_threads:
            return r
    return None


def write_traffic_summary(fetch_dir, write_dir, out, copy_n, grid_n):
    """Per-launch traffic of the two stage kernels from counter passes.  The
    copy kernel reads and writes 4*copy_n^2 bytes: the ratio to what each
    counter reports for it is that counter's calibration factor."""
    fetch, grid, fetch_g = _counter_means(fetch_dir, "FETCH_SIZE")
    write, _, write_g = _counter_means(write_dir, "WRITE_SIZE")
    copy_kib = 4.0 * copy_n * copy_n / 1024.0
    ff, wf = copy_kib / fetch["copy"], copy_kib / write["copy"]
    per = {k: {"fetch_kib": round(fetch[k], 1), "write_kib": round(write[k], 1),
               "bytes": round((fetch[k] * ff + write[k] * wf) * 1024.0),
               "tile_rows": rows_from_grid(grid[k], grid_n, 56 if k == "fused" else 60)}
           for k in STAGE_NAMES if k in fetch and k in write}
    # the fused step at every tile height the passes ran (the autotuner's
    # choice varies between balanced heights of equal speed)
    fused_by_rows = {}
    for (fam, g), fk in sorted(fetch_g.items()):
        if fam == "fused" and (fam, g) in write_g:
            wk = write_g[(fam, g)]
            fused_by_rows[str(rows_from_grid(g, grid_n, 56))] = {
                "fetch_kib": round(fk, 1), "write_kib": round(wk, 1), "bytes": round((fk * ff + wk * wf) * 1024.0)}
    unfused = [per[k]["bytes"] for k in ("fwd", "heun2") if k in per]
    summary = {"kernel_source_sha256": kernel_source_hash(), "grid": grid_n,
               "tile_rows": per["fwd"]["tile_rows"] if "fwd" in per else None,
               "copy_probe_n": copy_n,
               "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
               "copy_fetch_kib": round(fetch["copy"], 1), "copy_write_kib": round(write["copy"], 1),
               "stage": per,
               "bytes_per_launch": round(sum(unfused) / len(unfused)) if len(unfused) == 2 else None,
               "fused_bytes_per_launch": per["fused"]["bytes"] if "fused" in per else None,
               "fused_by_rows": fused_by_rows}
    with open(out, "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary))


def load_traffic(grid_n, precision, limiter, tile_rows, fused=False):
    """(bytes per launch, tile height the counters were taken at) for this
    workload, or None when no summary was measured on the current kernel
    sources and configuration.  Unfused: the average of the two stage
    launches, at the same tile height as the timed launches.  Fused: the
    one launch per step, at the timed height when the passes covered it,
    else at the profiled one (reported beside it)."""
    if precision != "fp32" or limiter != "superbee" or not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash() or t.get("grid") != grid_n:
        return None
    if fused:
        f = t.get("fused_by_rows", {}).get(str(tile_rows))
        if f:
            return f["bytes"], tile_rows
        f = t.get("stage", {}).get("fused")
        return (f["bytes"], f["tile_rows"]) if f else None
    if t.get("tile_rows") != tile_rows or not t.get("bytes_per_launch"):
        return None
    return t["bytes_per_launch"], t["tile_rows"]


def _make_instance(inst):
    a11, a12, v0 = inst.make()
    return a11, a12, v0


def batched_vs_plain(fdm, workloads, K, log, autotune=True):
    """The batched workload (384 instances, ~90M nodes): one K-step chunk as
    one graph of batched launches against one launch per instance per stage,
    and as one graph of batched fused Heun launches (one per step)."""
    import concurrent.futures as cf
    import numpy as np
    import torch

    insts = workloads.batched_instances()
    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1))
    import multiprocessing as mp
    # fresh worker interpreters: this process already holds a GPU context
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        arrays = list(ex.map(_make_instance, insts, chunksize=4))
    log("bench[batched]: generated %d instances in %.1f s" % (len(insts), time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    base11 = [torch.from_numpy(a[0]).to(dev) for a in arrays]
    base12 = [torch.from_numpy(a[1]).to(dev) for a in arrays]
    fields = [torch.from_numpy(a[2]).to(dev) if a[2] is not None else None for a in arrays]
    descs = [fdm.desc(i.nx, i.ny, limiter=i.limiter, cfl=0.4, v0=i.v0, v0_field=f) for i, f in zip(insts, fields)]
    nodes = sum(i.nx * i.ny for i in insts)
    stream = torch.cuda.current_stream()
    out = {}
    finals = {}
    rows = {}
    for sched in ("batched", "plain", "fused"):
        s11 = [b.clone() for b in base11]
        s12 = [b.clone() for b in base12]
        ctx = fdm.fdm_transport_init(descs, options={"schedule": sched}, stream=stream, keep=fields)
        if autotune:
            trials = fdm.fdm_autotune(ctx, s11, s12, trial_steps=2)
            log("bench[batched]: %s autotune: %s" % (sched, ", ".join("%d rows %.3f ms" % (
                t["tile_rows"], 1e3 * t["seconds_per_step"]) for t in trials)))
        rows[sched] = fdm.fdm_tile_rows(ctx, 0)
        if sched != "plain":
            fdm.fdm_run(ctx, s11, s12, K, K, history=False)      # capture + warm
        else:
            fdm.fdm_transport_step(ctx, s11, s12, 2)
        torch.cuda.synchronize()
        # restart from the same inputs for the timed chunk
        for a, b in zip(s11, base11):
            a.copy_(b)
        for a, b in zip(s12, base12):
            a.copy_(b)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if sched != "plain":
            fdm.fdm_run(ctx, s11, s12, K, K, history=False)
        else:
            fdm.fdm_transport_step(ctx, s11, s12, K)
        e1.record(stream)
        torch.cuda.synchronize()
        dt_s = e0.elapsed_time(e1) / 1000.0
        stats = fdm.fdm_transport_stats(ctx, s11, s12, allow_nonfinite=True)
        fdm.fdm_destroy(ctx)
        out[sched] = {"seconds": round(dt_s, 4), "cell_updates_per_s": round(nodes * K / dt_s, 1),
                      "tile_rows": rows[sched],
                      "nonfinite_instances": sum(1 for st in stats if st["nonfinite"])}
        finals[sched] = (s11, s12)
        log("bench[batched]: %s %d steps in %.3f s (%.3e cell-updates/s)" % (sched, K, dt_s, nodes * K / dt_s))
    def same(a, b):
        return all(torch.equal(x, y) for x, y in zip(finals[a][0], finals[b][0])) and \
            all(torch.equal(x, y) for x, y in zip(finals[a][1], finals[b][1]))
    return {"instances": len(insts), "nodes": nodes, "chunk_steps": K,
            "batched": out["batched"], "plain": out["plain"], "fused_batched": out["fused"],
            "speedup": round(out["plain"]["seconds"] / out["batched"]["seconds"], 3),
            "fused_speedup_vs_plain": round(out["plain"]["seconds"] / out["fused"]["seconds"], 3),
            "bitwise_equal": bool(same("batched", "plain")),
            "fused_bitwise_equal": bool(same("fused", "plain"))}


def coupled_leg(fdm, workloads, n_steps, log, n=512):
    """The coupled workload: a 512^2 layer with 20 seeded loops (plateaus
    +-0.2, erfc edges sigma 2, radii 20-80), a 4-voxel layer in a 512-voxel
    cell, mu = 1, nu = 0.3, threshold 0.01, mobility 1, strain rate 1e-3,
    CFL 0.4 with the step capped at 0.02; n_steps coupled steps (static
    solve, velocity law, adaptive step, transport, mean slip) in 10 chunks."""
    import torch
    phi, a11, a12 = workloads.plateau_rings(n, n, seed=4)
    dev = torch.device("cuda:0")
    t11, t12 = torch.from_numpy(a11).to(dev), torch.from_numpy(a12).to(dev)
    stream = torch.cuda.current_stream()
    ctx = fdm.fdm_transport_init(fdm.desc(n, n, limiter="minmod", cfl=0.4, v0=-1.0), stream=stream)
    L = fdm.loading(strain_rate13=1e-3, tau0=0.01, mobility=1.0, mu=1.0, lam=1.5, layer_h=4.0, cell_l3=512.0,
                    dt_max=0.02, eps13=0.0, phi_mean=float(phi.mean()))
    chunk = max(1, n_steps // 10)
    fdm.fdm_run(ctx, t11.clone(), t12.clone(), 20, 20, loading=L)    # plans, workspace, warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = fdm.fdm_run(ctx, t11, t12, n_steps, chunk, loading=L)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    fdm.fdm_destroy(ctx)
    log("bench[coupled]: %d coupled steps in %.3f s (%.1f us/step)" % (n_steps, sec, 1e6 * sec / n_steps))
    return {"grid": [n, n], "steps": n_steps, "seconds": round(sec, 4),
            "ms_per_step": round(1e3 * sec / n_steps, 4),
            "cell_updates_per_s": round(n * n * n_steps / sec, 1),
            "timing": "host wall clock over the call (step scalars stay on the device; one sync per chunk)",
            "stress_strain": [[round(r[0]["eps13"], 7), round(r[0]["sigma13"], 8), round(r[0]["phi_mean"], 8),
                               round(r[0]["vmax"], 6)] for r in hist],
            "stress_strain_columns": ["eps13", "sigma13", "phi_mean", "vmax"]}


def celerity_field_leg(fdm, workloads, K, log, n=4096, autotune=True):
    """The spatially varying celerity workload: 4096^2 diagonal bands (64
    bands, seed 3) under a Fourier-mode celerity field, minmod, Heun, CFL
    0.45.  State, stage buffer and field (320 MiB) exceed the 256 MB MALL, so
    this is the HBM-side figure.  The plain schedule (two stage launches per
    step, 48 B per node with the field) is timed beside the autotuned one,
    and a device-to-device copy of the same bytes per step as the practical
    streaming peak."""
    import torch
    a11, a12, v0 = workloads.bands_and_celerity(n, seed=3)
    dev = torch.device("cuda:0")
    tv = torch.from_numpy(v0).to(dev)
    stream = torch.cuda.current_stream()

    def timed(schedule, tune):
        t11, t12 = torch.from_numpy(a11).to(dev), torch.from_numpy(a12).to(dev)
        ctx = fdm.fdm_transport_init(fdm.desc(n, n, limiter="minmod", cfl=0.45, v0_field=tv),
                                     options={"schedule": schedule}, stream=stream, keep=[tv])
        sched = "plain" if schedule == "auto" else schedule   # untuned AUTO keeps the two stage launches
        if tune:
            trials = fdm.fdm_autotune(ctx, [t11], [t12], trial_steps=5)
            sched = min(trials, key=lambda t: t["seconds_per_step"])["schedule"]
        rows = fdm.fdm_tile_rows(ctx, 0)
        fdm.fdm_run(ctx, t11, t12, K, K)          # captures the chunk graph
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fdm.fdm_run(ctx, t11, t12, K, K)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1000.0)
        fdm.fdm_destroy(ctx)
        del t11, t12
        return sorted(times)[1], rows, sched

    t, rows, sched = timed("auto", autotune)
    tp, rows_p, _ = timed("plain", False)
    value = n * n * K / t
    plain = n * n * K / tp
    # reference: copy the bytes one unfused step must move at least (48 B per
    # node with the field) with a plain device-to-device copy
    nbytes = 48 * n * n
    src = torch.empty(nbytes // 8, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del src, dst
    alg = value * 20 / 1e9     # algorithmic bytes per cell-update with a field: 20
    unfused = value * 48 / 1e9
    plain_gbs = plain * 48 / 1e9
    log("bench[field]: %dx%d %.3e cell-updates/s (%d-row tiles, %s); plain %.3e (%.0f GB/s, %.2f of HBM peak); "
        "copy reference %.0f GB/s" % (n, n, value, rows, sched, plain, plain_gbs, plain_gbs / HBM_PEAK_GBS,
                                      copy_gbs))
    return {"grid": [n, n], "limiter": "minmod", "cfl": 0.45, "steps": K, "tile_rows": rows, "schedule": sched,
            "ms_per_step": round(1e3 * t / K, 4), "cell_updates_per_s": round(value, 1),
            "hbm_frac_algorithmic": round(alg / HBM_PEAK_GBS, 4),
            "unfused_stream_gbs": round(unfused, 1),
            "plain": {"tile_rows": rows_p, "ms_per_step": round(1e3 * tp / K, 4),
                      "cell_updates_per_s": round(plain, 1), "stream_gbs": round(plain_gbs, 1),
                      "hbm_frac": round(plain_gbs / HBM_PEAK_GBS, 4),
                      "bytes_per_cell_update": 48},
            "copy_reference_gbs": round(copy_gbs, 1),
            "unfused_stream_frac_of_copy": round(unfused / copy_gbs, 4),
            "timing": "HIP events around graph-replayed chunks, median of 3; copy: torch device copy of the same "
                      "48 B/node footprint"}


def fully_discrete_leg(fdm, workloads, n, K, limiter, log, autotune=True):
    """The same single-loop workload advanced by the paper's one-pass fully
    discrete scheme (one stage launch per step) at CFL 0.25."""
    import torch
    a11, a12 = workloads.ring(n, n, R=300.0 * n / 2048, sigma=6.0)
    dev = torch.device("cuda:0")
    t11, t12 = torch.from_numpy(a11).to(dev), torch.from_numpy(a12).to(dev)
    stream = torch.cuda.current_stream()
    ctx = fdm.fdm_transport_init(fdm.desc(n, n, limiter=limiter, cfl=0.25, v0=-1.0, time_order=1,
                                          scheme="fully_discrete"), stream=stream)
    if autotune:
        fdm.fdm_autotune(ctx, [t11], [t12], trial_steps=10)
    rows = fdm.fdm_tile_rows(ctx, 0)
    fdm.fdm_run(ctx, t11, t12, K, K)          # captures the chunk graph
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fdm.fdm_run(ctx, t11, t12, K, K)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1000.0)
    fdm.fdm_destroy(ctx)
    t = sorted(times)[1]
    log("bench[fd]: %d fully discrete steps, %.2f us/step, %d-row tiles" % (K, 1e6 * t / K, rows))
    return {"grid": [n, n], "limiter": limiter, "cfl": 0.25, "steps": K, "ms_per_step": round(1e3 * t / K, 5),
            "cell_updates_per_s": round(n * n * K / t, 1), "tile_rows": rows,
            "timing": "HIP events around graph-replayed chunks, median of 3"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--limiter", default="superbee")
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-rows", type=int, default=0, help="0: the library's default rule")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep --tile-rows instead of timing the candidate tilings first (fdm_autotune)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64_arith", "fp64"])
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--no-coupled", action="store_true", help="skip the coupled-run measurement")
    ap.add_argument("--no-fd", action="store_true", help="skip the fully-discrete-scheme measurement")
    ap.add_argument("--no-field", action="store_true", help="skip the 4096^2 celerity-field measurement")
    ap.add_argument("--schedule", default="auto", choices=["auto", "plain", "fused"],
                    help="launch schedule of the main workload (auto: the autotuner may pick fused)")
    ap.add_argument("--coupled-steps", type=int, default=5000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="N",
                    help="also run one single-stage (Euler) step on an N x N zero state: its copy-back is a "
                         "plain copy kernel reading and writing 4*N*N bytes per array, the byte reference for "
                         "the memory counters (use N >= 16384 so the arrays dwarf the caches)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no run: read rocprofv3 FETCH_SIZE and WRITE_SIZE counter CSVs of a profiled bench "
                         "run (with --copy-probe), write the per-launch traffic summary (--traffic-out)")
    ap.add_argument("--traffic-out", default=TRAFFIC_FILE)
    args = ap.parse_args()

    if args.traffic_from:
        write_traffic_summary(args.traffic_from[0], args.traffic_from[1], args.traffic_out,
                              args.copy_probe or 16384, args.n)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1911_03225_amd import fdm, workloads

    n, K, W = args.n, args.steps, args.warmup
    R, sigma, cfl = 300.0 * n / 2048, 6.0, 0.4
    log("bench: generating %dx%d ring" % (n, n))
    a11, a12 = workloads.ring(n, n, R=R, sigma=sigma)
    dev = torch.device("cuda:0")
    state = torch.float64 if args.precision == "fp64" else torch.float32
    t11 = torch.from_numpy(a11).to(dev).to(state)
    t12 = torch.from_numpy(a12).to(dev).to(state)
    stream = torch.cuda.current_stream()
    options = {"tile_rows": args.tile_rows, "precision": args.precision, "schedule": args.schedule}
    ctx = fdm.fdm_transport_init(fdm.desc(n, n, limiter=args.limiter, cfl=cfl, v0=-1.0), options=options,
                                 stream=stream)
    dt = fdm.fdm_transport_dt(ctx)
    tuning = None
    if not args.no_autotune:
        tuning = fdm.fdm_autotune(ctx, [t11], [t12], trial_steps=10)
        log("bench: autotune: %s" % ", ".join("%d rows %.2f us" % (t["tile_rows"], 1e6 * t["seconds_per_step"])
                                               for t in tuning))
    rows_used = fdm.fdm_tile_rows(ctx, 0)
    if tuning:
        sched_used = min(tuning, key=lambda t: t["seconds_per_step"])["schedule"]
    else:
        sched_used = "fused" if args.schedule == "fused" else "plain"
    fused = sched_used == "fused"

    log("bench: warmup %d steps + one captured chunk of %d (%d-row tiles, %s launches)"
        % (W, K, rows_used, sched_used))
    fdm.fdm_transport_step(ctx, t11, t12, W)
    fdm.fdm_run(ctx, t11, t12, K, K)          # captures the chunk graph
    torch.cuda.synchronize()

    times = []
    for r in range(args.repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        hist = fdm.fdm_run(ctx, t11, t12, K, K)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1000.0)
        log("bench: repeat %d: %.3f ms/step, sum_abs %.6e" % (r, 1e3 * times[-1] / K, hist[-1][0]["sum_abs"]))
    t_med = sorted(times)[len(times) // 2]
    cells = n * n
    value = cells * K / t_med
    ms_per_step = 1e3 * t_med / K
    # Two stage launches per step (first and second Heun stage, the same
    # kernel template), or one fused launch; the per-chunk diagnostics are
    # < 1% of the region.  Dominant kernel: the stage kernel, ALU-bound.
    stages_per_launch = 2 if fused else 1
    launches = K * 2 // stages_per_launch
    kernel_s = t_med / launches
    ops_per_launch = OPS_PER_NODE_STAGE * cells * stages_per_launch
    achieved = ops_per_launch / kernel_s / 1e12
    tr = load_traffic(n, args.precision, args.limiter, rows_used, fused)
    alg_bytes = BYTES_PER_CELL_STEP * cells * stages_per_launch // 2
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
                "traffic": tr[0] if tr else None,
                "traffic_tile_rows": tr[1] if tr else None,
                "traffic_vs_algorithmic": round(tr[0] / alg_bytes, 3) if tr else None,
                "kernel": "fused_kernel (both Heun stages)" if fused
                else "stage_kernel (first and second Heun stage)",
                "kernel_avg_us": round(1e6 * kernel_s, 2), "ops_per_launch": ops_per_launch,
                "hbm_bytes_per_launch": alg_bytes,
                "unfused_min_bytes_per_launch": 20 * cells * stages_per_launch,
                "hbm_achieved_gbs": round(alg_bytes / kernel_s / 1e9, 1),
                # measured L2-to-fabric bytes (counter passes) over this run's launch time;
                # at 2048^2 the working set sits in the 256 MB MALL, which serves much of it
                "fabric_achieved_gbs": round(tr[0] / kernel_s / 1e9, 1) if tr else None,
                "fabric_frac_of_hbm_peak": round(tr[0] / kernel_s / 1e9 / HBM_PEAK_GBS, 4) if tr else None,
                # the same launch counted in issued instructions: the node-stages
                # the step needs (halo lanes and rows left out) at the compiled
                # code's instruction count, over the issue peak
                "issue_view": {"valu_instr_per_node_stage": ISSUED_PER_NODE_STAGE,
                               "useful_issue_frac": round(ISSUED_PER_NODE_STAGE * cells * stages_per_launch
                                                          / kernel_s / 1e12 / ALU_PEAK_TOPS, 4)}}
    final = hist[-1][0]
    fdm.fdm_destroy(ctx)

    if args.copy_probe:
        m = args.copy_probe
        z11 = torch.zeros((m, m), dtype=torch.float32, device=dev)
        z12 = torch.zeros((m, m), dtype=torch.float32, device=dev)
        ctx1 = fdm.fdm_transport_init(fdm.desc(m, m, limiter=args.limiter, cfl=cfl, v0=-1.0, time_order=1),
                                      stream=stream)
        fdm.fdm_transport_step(ctx1, z11, z12, 1)
        torch.cuda.synchronize()
        fdm.fdm_destroy(ctx1)
        del z11, z12
        log("bench: copy probe: one Euler step on %dx%d, copy kernel of %d bytes per array" % (m, m, 4 * m * m))

    batched_leg = None
    if not args.no_batched:
        batched_leg = batched_vs_plain(fdm, workloads, args.batched_steps, log, autotune=not args.no_autotune)

    coupled_run_leg = None
    if not args.no_coupled:
        coupled_run_leg = coupled_leg(fdm, workloads, args.coupled_steps, log)

    field_leg = None
    if not args.no_field:
        field_leg = celerity_field_leg(fdm, workloads, 100, log, autotune=not args.no_autotune)

    fd = None
    if not args.no_fd:
        fd = fully_discrete_leg(fdm, workloads, n, K, args.limiter, log, autotune=not args.no_autotune)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        P = oracle.Problem(n, n, limiter=args.limiter, v0=-1.0, dt=dt)
        c11, c12 = a11.astype(np.float64), a12.astype(np.float64)
        steps, t0 = 0, time.perf_counter()
        while True:
            c11, c12 = oracle.run(P, c11, c12, 1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or steps >= 2000:
                break
        cpu = {"value": round(cells * steps / el, 1), "unit": "cell-updates/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": "first %d steps of the same %dx%d workload (FP64, OpenMP over rows), %.1f s" %
                         (steps, n, n, el)}
        log("bench: oracle %d steps in %.1f s on %d threads" % (steps, el, oracle.max_threads()))

    out = {
        "metric": "transport cell-updates/s", "value": round(value, 1), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": {"fp32": "f32", "fp64_arith": "f64 arithmetic, f32 state", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "single loop %dx%d (ring R=%g sigma=%g), LAW v0=-1, %s, Heun, CFL %g"
                               % (n, n, R, sigma, args.limiter, cfl),
                   "grid": [n, n], "limiter": args.limiter, "cfl": cfl, "dt": dt, "time_order": 2,
                   "chunk_steps": K, "tile_rows": rows_used, "schedule": sched_used,
                   "tiling": "autotuned" if tuning else ("fixed" if args.tile_rows else "default rule"),
                   "precision": args.precision},
        "hbm_frac_algorithmic": round(value * BYTES_PER_CELL_STEP / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_vs_plain": batched_leg,
        "coupled": coupled_run_leg,
        "fully_discrete": fd,
        "celerity_field_4096": field_leg,
        "final_stats": {"step": final["step"], "sum_abs": final["sum_abs"], "max_norm": final["max_norm"],
                        "drift11": final["drift11"], "drift12": final["drift12"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
