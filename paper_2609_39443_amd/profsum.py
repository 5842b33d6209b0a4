"""Summaries of rocprofv3 output for the canopy bench workload (256^3 cells,
2000 stems, FP32-split, batched graph step): a per-kernel time table, a
per-kernel counter table, and the HBM traffic per launch that bench.py
reports beside its roofline figure.

The raw output comes from these runs, from the repository root with
TMPDIR=/tmp (each counter group in a pass of its own):

  rocprofv3 --kernel-trace --stats --output-format csv -d OUT/prof -o canopy -- <BENCH>
  rocprofv3 --pmc <SQ counters> --output-format csv -d OUT/pmc -o sq -- <BENCH_PMC>
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/pmc -o fetch -- <BENCH_PMC> --copy-probe-mb 1024
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/pmc -o write -- <BENCH_PMC> --copy-probe-mb 1024
  rocprofv3 --pmc <LDS counters> --output-format csv -d OUT/pmc -o lds -- <BENCH_PMC>

then

  python -m paper_2609_39443_amd.profsum OUT profiles

HBM bytes are calibrated on the plain 1 GiB device copy that
`--copy-probe-mb 1024` runs first: the factor for each counter is the bytes
the copy moves divided by what that counter reads for it.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

BENCH = "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-fp64 --no-extra --no-autotune"
BENCH_PMC = "python3 bench.py --steps 2 --warmup 0 --no-cpu-baseline --no-fp64 --no-extra --no-autotune"
SQ = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_INSTS_SMEM SQ_WAIT_INST_ANY "
      "SQ_BUSY_CYCLES SQ_WAVE_CYCLES")
LDS = ("SQ_LDS_BANK_CONFLICT SQ_LDS_ADDR_CONFLICT SQ_LDS_IDX_ACTIVE SQ_INSTS_LDS SQ_ACTIVE_INST_LDS "
       "SQ_WAIT_INST_LDS")


def commands(out: str) -> dict:
    """The rocprofv3 runs whose output (under `out`) the summaries read."""
    return {
        "trace": (f"timeout -s KILL 300 rocprofv3 --kernel-trace --stats --output-format csv -d {out}/prof "
                  f"-o canopy -- {BENCH}"),
        "sq": f"timeout -s KILL 240 rocprofv3 --pmc {SQ} --output-format csv -d {out}/pmc -o sq -- {BENCH_PMC}",
        "fetch": (f"timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/pmc -o fetch -- "
                  f"{BENCH_PMC} --copy-probe-mb 1024"),
        "write": (f"timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/pmc -o write -- "
                  f"{BENCH_PMC} --copy-probe-mb 1024"),
        "lds": f"timeout -s KILL 240 rocprofv3 --pmc {LDS} --output-format csv -d {out}/pmc -o lds -- {BENCH_PMC}",
    }
WORKLOAD = "canopy 256^3 / 2000 stems, FP32-split graph step"
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_KIB = 1024 * 1024  # the 1 GiB calibration copy, each way
# kernels whose counters go into the traffic table (the per-step hot path)
HOT = ("k_weights", "k_weights64", "k_weights_int", "k_weights_int64", "k_spread", "k_sample", "k_tile_merge",
       "k_chunk_tiles", "k_emit_scatter",
       "k_chunk_boxes", "k_points_prep", "k_items", "k_drag", "k_norm")


def hot(name: str) -> bool:
    """A per-step kernel of the table (template arguments ignored)."""
    return name.split("<")[0] in HOT


def source_hash() -> str:
    """sha256 (first 16 hex) of the kernel sources, in file-name order; the
    same digest bench.py checks before it reports the traffic figure."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_39443_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("alp::", "").strip()


def trace_table(stats_csv: str) -> str:
    rows = []
    for r in csv.DictReader(open(stats_csv)):
        rows.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                     float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[1] * x[2])
    out = [f"{'kernel':44s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for k, n, a, lo, hi, p in rows[:24]:
        out.append(f"{k[:44]:44s} {n:6d} {a:10.1f} {lo:10.1f} {hi:10.1f} {p:6.2f}")
    return "\n".join(out)


def counters(path: str) -> dict:
    """kernel -> mean over dispatches of each counter, plus mean duration (ns),
    dispatch count and grid size in waves of 64."""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    dur = collections.defaultdict(dict)
    grid = {}
    for r in csv.DictReader(open(path)):
        k = short(r["Kernel_Name"])
        d = int(r["Dispatch_Id"])
        per[k][d][r["Counter_Name"]] += float(r["Counter_Value"])
        dur[k][d] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        grid[k] = int(r["Grid_Size"])
    out = {}
    for k, ds in per.items():
        acc = collections.defaultdict(list)
        for c in ds.values():
            for n, v in c.items():
                acc[n].append(v)
        out[k] = {n: sum(v) / len(v) for n, v in acc.items()}
        out[k]["_n"] = len(ds)
        out[k]["_dur_ns"] = sum(dur[k].values()) / len(dur[k])
        out[k]["_waves"] = (grid[k] + 63) // 64
    return out


def copy_reading(path: str, counter: str) -> float:
    """The counter's reading for the largest device copy in the run (the
    calibration copy)."""
    best = 0.0
    per = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if COPY_KERNEL in r["Kernel_Name"] and r["Counter_Name"] == counter:
            per[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
    for v in per.values():
        best = max(best, v)
    if best <= 0:
        raise SystemExit(f"no calibration copy found in {path}")
    return best


def main(argv):
    if len(argv) != 3:
        raise SystemExit("usage: python -m paper_2609_39443_amd.profsum <rocprof out dir> <profiles dir>")
    src, dst = argv[1], argv[2]
    cmds = commands(src.rstrip("/"))
    again = f"python -m paper_2609_39443_amd.profsum {src} {dst}"
    tag = "canopy_256cubed_2000stems"
    sh = source_hash()
    # kernel trace
    stats = os.path.join(src, "prof", "canopy_kernel_stats.csv")
    head = (f"Kernel trace statistics: {WORKLOAD}.\n"
            "221,489 actuator points, 8.96M band cells, 25.8M pairs.\n"
            f"Kernel sources: csrc hash {sh} (sha256 of paper_2609_39443_amd/csrc/*.hip|*.h, first 16 hex).\n"
            "Device: one MI355X (gfx950).  The calls count every execution of the step in the run: the first\n"
            "sizing/capturing call, the warmup and timed graph replays, and the per-stage profile steps\n"
            "(alp_step_profile: unforked, one stream).  In the graph, sampling and drag run on a second stream\n"
            "beside the segment binning, so kernels that overlap k_sample show inflated maxima.  The mesh\n"
            "binning kernels run once (alp_bin_cells).\n\n"
            "Command (from the repository root, TMPDIR=/tmp):\n  " + cmds["trace"] + "\n"
            f"Summarised with: {again}\n\n")
    with open(os.path.join(dst, f"{tag}_kernel_trace.txt"), "w") as fh:
        fh.write(head + trace_table(stats) + "\n")
    # counters
    pmc = os.path.join(src, "pmc")
    fpath, wpath = os.path.join(pmc, "fetch_counter_collection.csv"), os.path.join(pmc, "write_counter_collection.csv")
    sq = counters(os.path.join(pmc, "sq_counter_collection.csv"))
    fe, wr = counters(fpath), counters(wpath)
    cf, cw = copy_reading(fpath, "FETCH_SIZE"), copy_reading(wpath, "WRITE_SIZE")
    ff, wf = COPY_KIB / cf, COPY_KIB / cw
    traffic = {"source_hash": sh, "n_cells": 256 ** 3, "stems": 2000, "workload": WORKLOAD,
               "fetch_factor": ff, "write_factor": wf, "copy_fetch_kib": cf, "copy_write_kib": cw,
               "kernels": {}}
    lines = [f"{'kernel':16s} {'disp':>5s} {'avg_us':>8s} {'waves':>7s} {'VALU':>12s} {'LDS':>10s} {'SALU':>11s} "
             f"{'fetchKiB':>10s} {'writeKiB':>10s} {'HBM_MB':>8s} {'GB/s':>8s}"]
    for k in sorted((k for k in fe if hot(k) and k in wr), key=lambda k: -fe[k]["_dur_ns"]):
        fk, wk = fe[k]["FETCH_SIZE"], wr[k]["WRITE_SIZE"]
        b = (fk * ff + wk * wf) * 1024.0
        dur = 0.5 * (fe[k]["_dur_ns"] + wr[k]["_dur_ns"])
        traffic["kernels"][k] = {"fetch_kib": fk, "write_kib": wk, "bytes_per_launch": b, "avg_ns": dur}
        s = sq.get(k, {})
        if "SQ_INSTS_VALU" in s:
            # VALU wave instructions per dispatch and the SQ pass's own mean duration
            traffic["kernels"][k]["valu_insts"] = s["SQ_INSTS_VALU"]
            traffic["kernels"][k]["sq_avg_ns"] = s["_dur_ns"]
        lines.append(f"{k:16s} {fe[k]['_n']:5d} {dur / 1e3:8.1f} {fe[k]['_waves']:7d} "
                     f"{s.get('SQ_INSTS_VALU', 0):12.0f} {s.get('SQ_INSTS_LDS', 0):10.0f} "
                     f"{s.get('SQ_INSTS_SALU', 0):11.0f} {fk:10.0f} {wk:10.0f} {b / 1e6:8.1f} {b / dur:8.1f}")
    head = (f"Hardware counters per dispatch (mean over dispatches): {WORKLOAD}.\n"
            f"Kernel sources: csrc hash {sh}.  Device: one MI355X (gfx950).\n\n"
            "Commands (from the repository root, TMPDIR=/tmp), one pass per counter group:\n  "
            + "\n  ".join(cmds[k] for k in ("sq", "fetch", "write", "lds")) + "\n"
            f"Summarised with: {again}\n\n"
            f"Calibration: the 1 GiB device copy (--copy-probe-mb 1024, {COPY_KERNEL}) reads\n"
            f"FETCH_SIZE = {cf:.0f} KiB and WRITE_SIZE = {cw:.0f} KiB for {COPY_KIB:,} KiB moved each way,\n"
            f"so HBM bytes = FETCH_SIZE x {ff:.3f} + WRITE_SIZE x {wf:.3f} (KiB).\n\n")
    tail = ("\nHBM_MB = FETCH_SIZE x fetch factor + WRITE_SIZE x write factor (KiB -> MB); GB/s = HBM_MB over the\n"
            "mean duration of the same two passes.  VALU/LDS/SALU are instruction counts per dispatch (SQ pass).\n")
    # LDS pass: bank conflicts against the cycles the LDS was busy
    lpath = os.path.join(pmc, "lds_counter_collection.csv")
    if os.path.exists(lpath):
        ld = counters(lpath)
        tail += ("\nLDS counters per dispatch (the fourth pass above):\n"
                 f"{'kernel':16s} {'LDS_insts':>11s} {'LDS_active':>12s} {'bank_confl':>11s} {'addr_confl':>11s} "
                 f"{'confl/active':>12s}\n")
        for k in sorted((k for k in ld if hot(k) and ld[k].get("SQ_INSTS_LDS", 0) > 0),
                        key=lambda k: -ld[k].get("SQ_LDS_IDX_ACTIVE", 0)):
            c = ld[k]
            act = c.get("SQ_LDS_IDX_ACTIVE", 0.0)
            bc = c.get("SQ_LDS_BANK_CONFLICT", 0.0)
            tail += (f"{k:16s} {c.get('SQ_INSTS_LDS', 0):11.0f} {act:12.0f} {bc:11.0f} "
                     f"{c.get('SQ_LDS_ADDR_CONFLICT', 0):11.0f} {(bc / act if act else 0.0):12.3f}\n")
        tail += ("LDS_active = SQ_LDS_IDX_ACTIVE (cycles the LDS served indexed operations), bank_confl =\n"
                 "SQ_LDS_BANK_CONFLICT (cycles stalled on bank conflicts), both summed over the device per dispatch.\n")
    with open(os.path.join(dst, f"{tag}_pmc.txt"), "w") as fh:
        fh.write(head + "\n".join(lines) + "\n" + tail)
    with open(os.path.join(dst, "traffic.json"), "w") as fh:
        json.dump(traffic, fh, indent=1)
        fh.write("\n")
    print(f"wrote {tag}_kernel_trace.txt, {tag}_pmc.txt, traffic.json (source hash {sh})")


if __name__ == "__main__":
    main(sys.argv)
