#!/usr/bin/env python3
"""Benchmark of the actuator-line coupling step on one MI355X.

A step is one pass of the whole operator (segment binning, upstream sampling,
drag and relaxation, nodal weights, normalisation, spreading, conservation
check) over the canopy workload: 256^3 uniform cells (h = 4 mm, 16.8M cells),
2000 straight stems of 20..200 CVs (about 220k actuator points) with
overlapping kernels, all stems in one persistent launch per stage, the step
captured in a hipGraph and replayed.  Inputs are seeded synthetic arrays,
resident in HBM before timing starts.

Prints one JSON line: actuator points/s of the FP32-split batched step (the
headline), plus cell-updates/s, the algorithmic HBM rate, the all-FP64 and the
plain (unbatched, uncaptured) FP64 timings, live per-stage timings, the
roofline of the dominant kernel and the oracle's CPU baseline on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0       # MI355X HBM3E
VALU_PEAK_TOPS = 39.32       # 256 CU x 64 lanes x 2.4 GHz (non-packed FP32 / FP64 lane-ops)
N_SIMD = 256 * 4             # SIMDs: 4 per CU, 16 lanes each
CLOCK_GHZ = 2.4
VALU_CYCLES_PER_WAVE_INST = 4  # a wave64 VALU instruction on a 16-lane SIMD
# Algorithmic bytes the method itself moves per band cell over a whole step:
# the centre and volume read by the weights pass and again by the spread pass
# (centre FP32 in the split precision, FP64 otherwise; volume FP64), the
# source written (24 B) and the 4-byte cell index of the scatter.
BYTES_PER_BAND_CELL = {"split": 2 * (12 + 8) + 24 + 4, "fp64": 2 * (24 + 8) + 24 + 4}   # 68, 92
BYTES_PER_POINT = 272        # P, e_t, Pdot (72) + d, L, eps (24) + 2 velocity gathers (48)
                             # + f, U_s, P_s, w (80) + f_hat written and read (48)
# weights pass alone: centre + volume of each band cell
BYTES_WEIGHTS_PER_BAND_CELL = {"split": 12 + 8, "fp64": 24 + 8}
OPS_WEIGHTS_PER_PAIR = 50          # foot of eq. 21, eps_j, cutoff, eta of eq. 22, a0 a1, a V (lane-ops)
STAT_REPLAYS = 100                 # replays behind the per-step median and percentiles


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per mesh edge (default 256)")
    ap.add_argument("--stems", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stems", type=int, default=600,
                    help="stems in the oracle's timed sample: the stems rooted nearest the x = 0 "
                         "side of the canopy (a few seconds of CPU work per run)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle leg (0: the host's CPU share, at most 16)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison runs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary measurements (wave flume, batched scenarios, jittered net)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the headline at the default launch shape only (no ALP_AUTOTUNE search: "
                         "for profiler runs, whose per-kernel averages would otherwise mix candidate shapes)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def counters_from_profiles(kernel, n_cells, n_stems):
    """The committed rocprofv3 counter summary of `kernel` (HBM bytes per
    launch, VALU instructions, durations), if it was taken on the current
    sources and this workload; else an empty dict."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    try:
        t = json.load(open(p))
    except Exception:
        return {}
    from paper_2609_39443_amd.profsum import source_hash
    if t.get("source_hash") != source_hash() or t.get("n_cells") != n_cells or t.get("stems") != n_stems:
        return {}
    return t.get("kernels", {}).get(kernel) or {}


def measure_graph(alp, torch, np, wls, prec, steps, warmup, autotune=False):
    """Device copies of `wls`, one batched graph-captured step over all of
    them: ms per step and the diagnostics of every case.  With autotune, every
    case's cells are first rebinned with the batch binning autotuner and the
    launch shape is chosen by ALP_AUTOTUNE; the choices are returned."""
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = alp.Context(0)
    keep, cases, info = [], [], {}
    try:
        for wl in wls:
            C, V, U = dev(wl["C"]), dev(wl["V"]), dev(wl["U"])
            mesh = ctx.bin_cells(C, V, wl.get("box"))
            beams = alp.DeviceBeams(wl["beams"])
            f = torch.zeros(beams.n_points, 3, dtype=torch.float64, device="cuda")
            S = torch.zeros_like(C)
            keep.append((C, V, U, beams, f, S))
            cases.append(alp.alp_case(mesh, U.data_ptr(), beams.struct, alp.make_params(wl["params"], prec),
                                      None, f.data_ptr(), S.data_ptr(), None, None, None, None, None))
        flags = alp.USE_GRAPH
        alp.alp_set_tuning(ctx.h)
        if autotune:
            t0 = time.perf_counter()
            out = alp.alp_autotune_binning(ctx.h, cases, [k[0] for k in keep], [k[1] for k in keep],
                                           [wl.get("box") for wl in wls], reps=2)
            ctx.meshes.extend(out["meshes"])
            for c, m in zip(cases, out["meshes"]):
                c.mesh = m
            info["binning"] = {"bin_scale": out["scale"], "tile_bins": out["tile_bins"]}
            flags |= alp.AUTOTUNE
            alp.alp_step_batched(ctx.h, cases, flags)
            info["tuning"] = alp.alp_get_tuning(ctx.h)
            info["autotune_s"] = time.perf_counter() - t0
            flags = alp.USE_GRAPH
        alp.alp_step_batched(ctx.h, cases, flags)
        for _ in range(warmup):
            alp.alp_step_batched(ctx.h, cases, flags)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            alp.alp_step_batched(ctx.h, cases, flags)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        alp.alp_invalidate(ctx.h)
        diags = [ctx.diag(i) for i in range(len(cases))]
    finally:
        ctx.close()
    return dt, diags, info


def host_description():
    """Host core count and CPU model (the oracle's timings depend on them)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity_cpus": share, "cpu_model": model}


def beam_boxes(beams):
    """Per beam, the AABB of its points inflated by 3 eps_max plus its longest
    segment: every cell the beam reaches lies inside."""
    import numpy as np
    off = beams["offsets"]
    nb = len(off) - 1
    lo = np.full((nb, 3), np.inf)
    hi = np.full((nb, 3), -np.inf)
    for b in range(nb):
        P = beams["P"][off[b]:off[b + 1]]
        if P.shape[0] == 0:
            continue
        seg = np.linalg.norm(np.diff(P, axis=0), axis=1).max() if P.shape[0] > 1 else 0.0
        r = 3.0 * beams["eps"][off[b]:off[b + 1]].max() + seg + 1e-9
        lo[b], hi[b] = P.min(0) - r, P.max(0) + r
    return lo, hi


def cpu_baseline(wl, got, n_stems, n_cells):
    """The oracle (plain FP64 C, grid mode) on a bounded sample of the
    workload: the n_stems stems rooted nearest x = 0, over the full mesh, one
    whole step (sample, drag, project; the grid is built beforehand and not
    timed).  Median of three runs on one thread, and of three runs on all of
    the host's CPU share (the sample's stems in contiguous blocks, one oracle
    call per thread; per-point outputs depend only on their own beam and the
    sources superpose over beams, so the blocks are summed in block order).
    The first single-thread run also gives the accuracy of the GPU outputs on
    that sample: w of the sampled nodes, and S at band cells that only sampled
    stems can reach."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle
    from paper_2609_39443_amd import workloads as W

    host = host_description()
    beams = wl["beams"]
    off = beams["offsets"]
    nb = len(off) - 1
    order = np.argsort(beams["P"][off[:-1], 0], kind="stable")
    pick = sorted(order[:min(n_stems, nb)].tolist())
    sub = W.subset_beams(beams, pick)
    npt = int(sub["P"].shape[0])
    t0 = time.perf_counter()
    om = oracle.Mesh(wl["C"], wl["V"], wl.get("box"), oracle.GRID)
    t_grid = time.perf_counter() - t0
    log(f"oracle CPU baseline: {len(pick)} stems ({npt} points), grid built in {t_grid:.1f} s")
    singles, ref = [], None
    for _ in range(3):
        t = time.perf_counter()
        r = oracle.step(om, wl["U"], sub, wl["params"])
        singles.append(time.perf_counter() - t)
        ref = ref or r
    threads = host["affinity_cpus"] or 1
    threads = max(1, min(16, threads))
    per = -(-len(pick) // threads)
    blocks = [pick[i:i + per] for i in range(0, len(pick), per)]
    subs = [W.subset_beams(beams, b) for b in blocks]
    multi = []
    with ThreadPoolExecutor(max_workers=len(subs)) as ex:
        for _ in range(3):
            t = time.perf_counter()
            parts = list(ex.map(lambda sb: oracle.step(om, wl["U"], sb, wl["params"]), subs))
            Ssum = parts[0]["S"].copy()
            for q in parts[1:]:
                Ssum += q["S"]
            multi.append(time.perf_counter() - t)
            del parts, Ssum
    ts, tm = float(np.median(singles)), float(np.median(multi))
    cpu = {"value": npt / ts, "unit": "points/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(pick)} of {nb} stems (the ones rooted nearest x = 0; {npt} points) on the full "
                     f"{n_cells}-cell mesh, one FP64 step (sample, drag, project), grid mode, median of 3 "
                     f"runs of {ts:.2f} s",
           "seconds": singles, "pairs": int(ref["diag"]["n_pairs"]),
           "all_cores": {"value": npt / tm, "unit": "points/s", "cores": len(subs), "seconds": multi,
                         "how": "contiguous beam blocks, one oracle call per thread, sources summed in block order"},
           "grid_build_s": t_grid, **host}
    log(f"oracle: 1 thread {ts:.2f} s, {len(subs)} threads {tm:.2f} s")
    # accuracy on the sample
    idx = np.concatenate([np.arange(off[b], off[b + 1]) for b in pick])
    zw = ref["w"] == 0
    rng = np.random.default_rng(11)
    acc = {"sample": f"w of the {npt} sampled nodes; S at band cells reached only by sampled stems"}
    # band cells of the sample that no other stem can reach
    band = np.nonzero(np.any(ref["S"] != 0, axis=1))[0]
    cand = rng.choice(band, size=min(3000, band.size), replace=False)
    lo, hi = beam_boxes(beams)
    other = np.ones(nb, dtype=bool)
    other[pick] = False
    X = wl["C"][cand]
    reach = np.all((X[:, None, :] >= lo[None, other]) & (X[:, None, :] <= hi[None, other]), axis=2)
    cells = np.sort(cand[~reach.any(axis=1)][:400])
    for tag, g in got.items():
        gw = g["w"][idx]
        werr = float(np.max(np.abs(gw[~zw] - ref["w"][~zw]) / ref["w"][~zw])) if np.any(~zw) else 0.0
        Sg, Sr = g["S"][cells], ref["S"][cells]
        nr = np.linalg.norm(Sr, axis=1)
        e_cell = float(np.max(np.linalg.norm(Sg - Sr, axis=1)) / np.max(nr)) if cells.size else None
        big = nr > 1e-6 * np.max(nr) if cells.size else np.zeros(0, bool)
        e_rel = float(np.max(np.linalg.norm(Sg - Sr, axis=1)[big] / nr[big])) if np.any(big) else None
        acc[tag] = {"e_cell": e_cell, "e_cell_percell_rel_max": e_rel, "w_rel_max": werr,
                    "cells_checked": int(cells.size), "tol_e_cell": 1e-5 if tag == "split" else 1e-12}
    log(f"accuracy on the oracle sample: {acc}")
    return cpu, acc


def _integrated(wl):
    wl["params"] = dict(wl["params"], proj_mode="integrated")
    return wl


def secondary(alp, W, torch, np, steps):
    """The other workloads at their full sizes, FP32-split and all-FP64."""
    out = {}
    specs = [
        ("wave_flume", lambda: [W.wave_flume(snapshot=0)],
         "1,987,200 graded cells, one bent stem of 100 CVs"),
        ("jittered_net", lambda: [W.jittered_net()],
         "8M jittered cells in random order, 700 x 700-strand net of 499,800 points"),
        ("batched_scenarios", lambda: [W.scenario(c) for c in range(64)],
         "64 cases of 0.5M-4M cells and 1-500 stems of 20-300 CVs in one graph step"),
        ("canopy_integrated", lambda: [_integrated(W.canopy(n=256, n_stems=2000))],
         "the headline canopy (256^3 cells, 2000 stems) under the segment-integrated projection "
         "(a Gaussian integrated along every segment within the cutoff); pairs are (cell, segment)"),
    ]
    tuned = {"jittered_net", "batched_scenarios"}
    for name, make, desc in specs:
        t0 = time.time()
        wls = make()
        npnt = sum(wl["beams"]["P"].shape[0] for wl in wls)
        ncell = sum(wl["C"].shape[0] for wl in wls)
        log(f"{name}: {len(wls)} case(s), {ncell} cells, {npnt} points ({time.time() - t0:.1f} s to generate)")
        r = {"workload": desc, "n_cases": len(wls), "n_cells": ncell, "n_points": npnt}
        # the batched scenarios are timed over 100 replays, the others over `steps`
        nsteps = 100 if name == "batched_scenarios" else steps
        r["replays"] = nsteps
        legs = [("split", alp.PREC_FP32_SPLIT, False), ("fp64", alp.PREC_FP64, False)]
        if name in tuned:
            legs += [("split_autotuned", alp.PREC_FP32_SPLIT, True), ("fp64_autotuned", alp.PREC_FP64, True)]
        for tag, prec, auto in legs:
            dt, diags, info = measure_graph(alp, torch, np, wls, prec, nsteps, 2, autotune=auto)
            pairs = sum(int(d["n_pairs"]) for d in diags)
            r[f"{tag}_ms_per_step"] = dt * 1e3
            r[f"{tag}_points_per_s"] = npnt / dt
            r[f"{tag}_cell_updates_per_s"] = pairs / dt
            r[f"{tag}_max_cons_rel_err"] = max(float(d["cons_rel_err"]) for d in diags
                                               if int(d["n_zero_weight"]) == 0) if any(
                int(d["n_zero_weight"]) == 0 for d in diags) else None
            if info:
                r[f"{tag}_choice"] = info
            r["n_pairs"] = pairs
            r["n_band_cells"] = sum(int(d["n_band_cells"]) for d in diags)
            r["n_overflow"] = sum(int(d["n_overflow"]) for d in diags)
            r["n_guard_fp64"] = sum(int(d.get("n_guard_fp64", 0)) for d in diags)
            log(f"{name} {tag}: {dt * 1e3:.3f} ms/step {info if info else ''}")
        r["speedup_split_vs_fp64"] = r["fp64_ms_per_step"] / r["split_ms_per_step"]
        if name in tuned:
            r["speedup_autotuned_split"] = r["split_ms_per_step"] / r["split_autotuned_ms_per_step"]
        out[name] = r
        del wls
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU build: the coupling operator runs on one MI355X; "
                                   "--gpus must be 1 (the multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_39443_amd import alp
    from paper_2609_39443_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    alp.load()
    if args.copy_probe_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters
        nel = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    wl = W.canopy(n=args.n, n_stems=args.stems)
    log(f"workload {wl['name']}: {wl['C'].shape[0]} cells, {wl['beams']['P'].shape[0]} points "
        f"({time.time() - t0:.1f} s to generate)")
    dev = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    C, V, U = dev(wl["C"]), dev(wl["V"]), dev(wl["U"])
    n_cells = C.shape[0]
    ctx = alp.Context(0)
    mesh = ctx.bin_cells(C, V)
    beams = alp.DeviceBeams(wl["beams"])
    npnt = beams.n_points
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")
    out = {k: z(npnt, 3) for k in ("f", "U_s", "P_s")}
    out["w"] = z(npnt)
    S = z(n_cells, 3)
    cell_s = torch.zeros(npnt, dtype=torch.int64, device="cuda")

    def case(prec):
        return alp.alp_case(mesh, U.data_ptr(), beams.struct, alp.make_params(wl["params"], prec), None,
                            out["f"].data_ptr(), S.data_ptr(), out["U_s"].data_ptr(),
                            out["w"].data_ptr(), out["P_s"].data_ptr(), None, None)

    def timed_graph(prec, steps, warmup, stat_reps=STAT_REPLAYS, autotune=False):
        """K replays timed by the host clock between two synchronisations, then
        `stat_reps` replays timed one by one with events on the caller's
        stream (each replay is ordered on it): median, p10, p90.  With
        autotune the first call chooses the launch shape (ALP_AUTOTUNE);
        otherwise the default shape is used."""
        cs = [case(prec)]
        alp.alp_set_tuning(ctx.h)
        first = alp.USE_GRAPH | (alp.AUTOTUNE if autotune else 0)
        alp.alp_step_batched(ctx.h, cs, first)   # (tunes,) sizes, runs and captures
        for _ in range(warmup):
            alp.alp_step_batched(ctx.h, cs, alp.USE_GRAPH)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            alp.alp_step_batched(ctx.h, cs, alp.USE_GRAPH)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(stat_reps + 1)]
        ev[0].record()
        for i in range(stat_reps):
            alp.alp_step_batched(ctx.h, cs, alp.USE_GRAPH)
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(stat_reps)])
        stats = {"replays": stat_reps, "median_ms": float(np.median(per)),
                 "p10_ms": float(np.percentile(per, 10)), "p90_ms": float(np.percentile(per, 90))}
        stats["tuning"] = alp.alp_get_tuning(ctx.h)
        alp.alp_invalidate(ctx.h)
        return dt, ctx.diag(0), stats

    def timed_plain(prec, steps, warmup):
        p = alp.make_params(wl["params"], prec)

        def one():
            alp.alp_sample(ctx.h, mesh, U, beams.struct, p, out["U_s"], out["P_s"], None, cell_s)
            alp.alp_drag(ctx.h, beams.struct, p, out["U_s"], cell_s, None, out["f"])
            alp.alp_spread(ctx.h, mesh, beams.struct, p, out["f"], S, out["w"], None)
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def host_outputs():
        torch.cuda.synchronize()
        return {"S": S.cpu().numpy(), "w": out["w"].cpu().numpy(), "f": out["f"].cpu().numpy()}

    # the default launch shape first, then the headline: FP32-split, batched
    # persistent launches, launch shape chosen by ALP_AUTOTUNE, graph replay
    log("timing the FP32-split graph step, default launch shape")
    t_def, d_def, st_def = timed_graph(alp.PREC_FP32_SPLIT, args.steps, args.warmup)
    log(f"default shape: {t_def * 1e3:.3f} ms/step")
    if args.no_autotune:
        t_split, diag, st_split = t_def, d_def, st_def
    else:
        log("timing the FP32-split graph step, autotuned launch shape")
        t_split, diag, st_split = timed_graph(alp.PREC_FP32_SPLIT, args.steps, args.warmup, autotune=True)
    got = {"split": host_outputs()}
    log(f"split: {t_split * 1e3:.3f} ms/step (median {st_split['median_ms']:.3f}, "
        f"p10 {st_split['p10_ms']:.3f}, p90 {st_split['p90_ms']:.3f}), diag {diag}")
    # live per-stage timings (HIP events on the stream the kernels run on)
    alp.alp_set_tuning(ctx.h, **st_split["tuning"])  # the stage timings use the chosen shape
    stage_runs = [alp.alp_step_profile(ctx.h, [case(alp.PREC_FP32_SPLIT)]) for _ in range(5)]
    stages = {k: float(np.median([r[k] for r in stage_runs])) for k in stage_runs[0]}
    log(f"stages (ms): {stages}")
    res = {}
    stages64 = None
    if not args.no_fp64:
        t64, d64, st64 = timed_graph(alp.PREC_FP64, max(3, args.steps // 2), 1, autotune=True)
        got["fp64"] = host_outputs()
        res["fp64_graph_ms_per_step"] = t64 * 1e3
        res["fp64_step_stats"] = st64
        res["fp64_cons_rel_err"] = d64["cons_rel_err"]
        alp.alp_set_tuning(ctx.h, **st64["tuning"])
        stage64 = [alp.alp_step_profile(ctx.h, [case(alp.PREC_FP64)]) for _ in range(3)]
        stages64 = {k: float(np.median([r[k] for r in stage64])) for k in stage64[0]}
        res["fp64_stages_ms"] = stages64
        alp.alp_set_tuning(ctx.h)  # the plain path: unbatched, uncaptured, default shape
        tp = timed_plain(alp.PREC_FP64, max(3, args.steps // 4), 1)
        res["plain_fp64_unbatched_ms_per_step"] = tp * 1e3
        res["speedup_split_vs_fp64_graph"] = t64 / t_split
        res["speedup_vs_plain_fp64"] = tp / t_split
        log(f"fp64 graph {t64 * 1e3:.3f} ms, plain fp64 {tp * 1e3:.3f} ms")

    n_band, n_pairs = int(diag["n_band_cells"]), int(diag["n_pairs"])
    bytes_step = n_band * BYTES_PER_BAND_CELL["split"] + npnt * BYTES_PER_POINT
    gbps = bytes_step / t_split / 1e9
    # dominant kernel: the weights pass (closest segment per pair, eq. 21-22)
    t_w = stages["weights"] * 1e-3
    bytes_w = n_band * BYTES_WEIGHTS_PER_BAND_CELL["split"]
    ach_w = bytes_w / t_w / 1e9
    prof_w = counters_from_profiles("k_weights", n_cells, args.stems)
    traffic = prof_w.get("bytes_per_launch")
    roofline = {"kernel": "k_weights", "bound": "hbm", "achieved": ach_w, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": ach_w / HBM_PEAK_GBPS, "traffic": traffic,
                "alg_bytes_per_band_cell": BYTES_WEIGHTS_PER_BAND_CELL["split"],
                "alg_bytes_per_launch": bytes_w, "avg_ms": stages["weights"],
                "traffic_over_alg": (traffic / bytes_w) if traffic else None}
    if stages64:
        b64 = n_band * BYTES_WEIGHTS_PER_BAND_CELL["fp64"]
        a64 = b64 / (stages64["weights"] * 1e-3) / 1e9
        roofline["fp64"] = {"kernel": "k_weights64", "alg_bytes_per_band_cell": BYTES_WEIGHTS_PER_BAND_CELL["fp64"],
                            "alg_bytes_per_launch": b64, "avg_ms": stages64["weights"], "achieved": a64,
                            "frac": a64 / HBM_PEAK_GBPS}
    # the same kernel against the VALU roof: it issues far more instructions
    # than the method's arithmetic needs, so this view is reported beside
    ops_w = n_pairs * OPS_WEIGHTS_PER_PAIR
    roofline_alu = {"kernel": "k_weights", "bound": "alu", "achieved": ops_w / t_w / 1e12,
                    "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s", "frac": ops_w / t_w / 1e12 / VALU_PEAK_TOPS,
                    "alg_ops_per_launch": ops_w}
    # issued, not algorithmic: the counted VALU wave instructions of the same
    # kernel (each holds a 16-lane SIMD for 4 cycles) over the SIMD cycles of
    # its counted duration at 2.4 GHz
    if prof_w.get("valu_insts") and prof_w.get("sq_avg_ns"):
        busy = prof_w["valu_insts"] * VALU_CYCLES_PER_WAVE_INST
        roofline_alu["issued_valu_frac"] = busy / (N_SIMD * CLOCK_GHZ * prof_w["sq_avg_ns"])

    cpu = accuracy = None
    if not args.no_cpu_baseline:
        cpu, accuracy = cpu_baseline(wl, got, args.cpu_stems, n_cells)

    extra = None
    if not args.no_extra:
        extra = secondary(alp, W, torch, np, max(3, args.steps // 4))

    line = {
        "metric": "actuator points/s per coupling step", "value": npnt / t_split, "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_split * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32-split",
        "data": "synthetic",
        "config": {"workload": f"canopy: {args.n}^3 uniform cells (h = 4 mm), {args.stems} stems of "
                               f"20-200 CVs, FP32-split, all stems in one persistent launch per stage, "
                               + ("default launch shape" if args.no_autotune else "launch shape chosen by ALP_AUTOTUNE")
                               + ", hipGraph replay", "n_cells": n_cells,
                   "n_points": npnt,
                   "n_band_cells": n_band, "n_pairs": n_pairs, "parallelism": "single GPU"},
        "cell_updates_per_s": n_pairs / t_split, "band_cells_per_s": n_band / t_split,
        "mesh_cells_per_s": n_cells / t_split, "step_stats": st_split,
        "default_shape_ms_per_step": t_def * 1e3, "default_shape_step_stats": st_def,
        "alg_bytes_per_band_cell": BYTES_PER_BAND_CELL["split"], "alg_bytes_per_point": BYTES_PER_POINT,
        "alg_bytes_per_step": bytes_step, "alg_hbm_gbps": gbps, "alg_hbm_frac": gbps / HBM_PEAK_GBPS,
        "cons_rel_err": diag["cons_rel_err"], "accuracy": accuracy, "stages_ms": stages, "roofline": roofline,
        "roofline_alu": roofline_alu,
        "cpu_baseline": cpu, **res,
        "other_workloads": extra,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
