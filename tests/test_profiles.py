"""Host-side checks of the rocprofv3 summary code that feeds the benchmark's
roofline fields: the counter CSV parser and the lookup of the committed
counter summary, which is used only when it was taken on the current kernel
sources and the same workload."""

import json

import bench
from paper_2609_39443_amd import profsum


def _write_counters(path, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
            "Start_Timestamp", "End_Timestamp"]
    with open(path, "w") as fh:
        fh.write(",".join(cols) + "\n")
        for r in rows:
            fh.write(",".join(str(r[c]) for c in cols) + "\n")


def test_counters_mean_over_dispatches(tmp_path):
    """Per kernel: the counter summed within a dispatch, then averaged over
    dispatches; mean duration, dispatch count and grid size in waves."""
    p = tmp_path / "sq_counter_collection.csv"
    rows = []
    for d, (v1, v2, dur) in enumerate([(10, 30, 100), (20, 40, 300)]):
        for v in (v1, v2):  # two rows of one counter in one dispatch are summed
            rows.append({"Dispatch_Id": d, "Kernel_Name": "alp::k_weights(alp::StepLaunch)",
                         "Grid_Size": 262144, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": v,
                         "Start_Timestamp": 1000, "End_Timestamp": 1000 + dur})
    _write_counters(p, rows)
    c = profsum.counters(str(p))
    assert set(c) == {"k_weights"}
    k = c["k_weights"]
    assert k["SQ_INSTS_VALU"] == ((10 + 30) + (20 + 40)) / 2
    assert k["_n"] == 2 and k["_dur_ns"] == 200 and k["_waves"] == 4096


def _summary(tmp_path, monkeypatch, source_hash, n_cells=256 ** 3, stems=2000):
    (tmp_path / "profiles").mkdir()
    t = {"source_hash": source_hash, "n_cells": n_cells, "stems": stems,
         "kernels": {"k_weights": {"bytes_per_launch": 1.0e9, "avg_ns": 8.0e5,
                                   "valu_insts": 3.0e8, "sq_avg_ns": 8.0e5}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(t))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


def test_summary_used_on_current_sources(tmp_path, monkeypatch):
    _summary(tmp_path, monkeypatch, profsum.source_hash())
    k = bench.counters_from_profiles("k_weights", 256 ** 3, 2000)
    assert k["bytes_per_launch"] == 1.0e9 and k["valu_insts"] == 3.0e8
    assert bench.counters_from_profiles("k_spread", 256 ** 3, 2000) == {}


def test_summary_ignored_when_stale(tmp_path, monkeypatch):
    _summary(tmp_path, monkeypatch, "0" * 16)
    assert bench.counters_from_profiles("k_weights", 256 ** 3, 2000) == {}


def test_summary_ignored_for_another_workload(tmp_path, monkeypatch):
    _summary(tmp_path, monkeypatch, profsum.source_hash(), stems=1000)
    assert bench.counters_from_profiles("k_weights", 256 ** 3, 2000) == {}


def test_missing_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_from_profiles("k_weights", 256 ** 3, 2000) == {}
