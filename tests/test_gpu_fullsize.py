"""GPU parity at full workload sizes, in the launch configuration bench.py
times (FP32-split, all beams in one batched step, hipGraph replay).

The oracle cannot redo a 16.8M-cell canopy step in seconds, but every output
it needs can be computed one by one on a subset:
  - U_s, P_s and f of a point depend only on its own beam (eq. 16-20);
  - w_k of a node depends only on its own beam and the mesh (Sec. 3.2.4:
    beams are normalised independently);
  - S_j of a cell depends only on the beams that reach it, so the oracle run
    with exactly the beams whose inflated AABB contains the sampled cells
    gives S_j exactly at those cells.
Tolerances as in test_gpu_parity: FP64 quantities 1e-12, FP32-split weights
and sources 1e-5, conservation 1e-12, integer decisions exact.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2609_39443_amd import alp  # noqa: E402
from paper_2609_39443_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def gu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    return gpu_util


@pytest.fixture(scope="module")
def ctx(gu):
    alp.load()
    c = alp.Context(0)
    yield c
    c.close()


def beams_reaching(beams, X):
    """Beams whose points' AABB, inflated by 3 eps_max + the longest segment,
    contains any of the points X (a superset of the beams that reach X)."""
    off = beams["offsets"]
    out = []
    for b in range(len(off) - 1):
        P = beams["P"][off[b]:off[b + 1]]
        if P.shape[0] == 0:
            continue
        seg = np.linalg.norm(np.diff(P, axis=0), axis=1).max() if P.shape[0] > 1 else 0.0
        r = 3.0 * beams["eps"][off[b]:off[b + 1]].max() + seg + 1e-9
        lo, hi = P.min(0) - r, P.max(0) + r
        if np.any(np.all((X >= lo) & (X <= hi), axis=1)):
            out.append(b)
    return out


def sampled_check(gu, wl, res, diag, prec, n_beam_sample, n_cells_sample, seed, region=None):
    from oracle import oracle
    tS = 1e-12 if prec == alp.PREC_FP64 else 1e-5
    rng = np.random.default_rng(seed)
    beams = wl["beams"]
    off = beams["offsets"]
    nb = len(off) - 1
    om = oracle.Mesh(wl["C"], wl["V"], wl.get("box"), oracle.GRID)
    # 1. per-beam quantities on a sample of beams
    pick = sorted(rng.choice(nb, size=min(n_beam_sample, nb), replace=False).tolist())
    sub = W.subset_beams(beams, pick)
    ref = oracle.step(om, wl["U"], sub, wl["params"])
    idx = np.concatenate([np.arange(off[b], off[b + 1]) for b in pick])
    assert np.array_equal(res["cell_a"][idx], ref["cell_a"])
    assert np.array_equal(res["cell_s"][idx], ref["cell_s"])
    assert np.array_equal(res["U_s"][idx], ref["U_s"])
    assert gu.normwise(res["P_s"][idx], ref["P_s"]) <= 1e-15
    assert gu.normwise(res["f"][idx], ref["f"]) <= 1e-12
    zw = ref["w"] == 0
    assert np.all(res["w"][idx][zw] == 0)  # nodes that catch no cell (R12)
    werr = float(np.max(np.abs(res["w"][idx][~zw] - ref["w"][~zw]) / ref["w"][~zw])) if np.any(~zw) else 0.0
    assert werr <= tS, werr
    # 2. sources at sampled cells (band cells and some outside the band)
    band = np.nonzero(np.any(res["S"] != 0, axis=1))[0]
    if region is not None:
        inr = np.all((wl["C"][band] >= region[0]) & (wl["C"][band] <= region[1]), axis=1)
        band = band[inr]
    cells = rng.choice(band, size=min(n_cells_sample, band.size), replace=False)
    quiet = rng.choice(wl["C"].shape[0], size=50, replace=False)
    cells = np.unique(np.concatenate([cells, quiet]))
    near = beams_reaching(beams, wl["C"][cells])
    sub2 = W.subset_beams(beams, near)
    ref2 = oracle.step(om, wl["U"], sub2, wl["params"])
    Sg, Sr = res["S"][cells], ref2["S"][cells]
    err = gu.normwise(Sg, Sr)
    assert err <= tS, err
    assert np.all(Sg[np.all(Sr == 0, axis=1)] == 0)
    # 3. the exact balance of the transferred force (eq. 14), unless nodes
    #    outside the mesh caught no cell (then their share is missing by design)
    if diag["n_zero_weight"] == 0:
        assert diag["cons_rel_err"] <= 1e-12, diag
    assert diag["n_overflow"] == 0 and diag["n_invalid"] == 0
    return {"w": float(werr), "S": float(err), "beams_for_S": len(near), "cells": int(cells.size)}


def run_graph(gu, ctx, wl, prec, replays=3):
    case = gu.GpuCase(ctx, wl, prec)
    flags = alp.USE_GRAPH
    gu.step_batched(ctx, [case], flags)
    for _ in range(replays):
        gu.step_batched(ctx, [case], flags)
    res = case.results()
    diag = ctx.diag(0)
    alp.alp_invalidate(ctx.h)
    return case, res, diag


def test_wave_flume_full_size(gu, ctx):
    """2M graded cells, one bent stem of 100 CVs: the oracle redoes the whole
    step, both snapshots, both precisions."""
    for snap in (0, 1):
        wl = W.wave_flume(snapshot=snap)
        ref = gu.oracle_step(wl)
        for prec in (alp.PREC_FP64, alp.PREC_FP32_SPLIT):
            gu.log(f"[full] wave flume s{snap} prec={prec}")
            case, res, diag = run_graph(gu, ctx, wl, prec)
            tS = 1e-12 if prec == alp.PREC_FP64 else 1e-5
            err = gu.compare(res, ref, diag, ref["diag"], tS, tS)
            gu.log(f"[full]   {err}")
            del case


def test_canopy_full_size_sampled(gu, ctx):
    """16.8M cells, 2000 stems, 221k points, 25.8M pairs: the bench workload."""
    wl = W.canopy(n=256, n_stems=2000)
    gu.log("[full] canopy 256^3 / 2000 stems, FP32-split graph")
    case, res, diag = run_graph(gu, ctx, wl, alp.PREC_FP32_SPLIT, replays=2)
    del case
    torch.cuda.empty_cache()
    out = sampled_check(gu, wl, res, diag, alp.PREC_FP32_SPLIT, n_beam_sample=12,
                        n_cells_sample=120, seed=5)
    gu.log(f"[full]   {out}")


def test_jittered_net_full_size_sampled_and_permutation(gu, ctx):
    """8M jittered cells in random order, a 700 x 700-strand net (499,800
    points, ~46 strands per band cell); sampled parity on a patch, and bitwise
    identical results under another random permutation of the cells."""
    wl = W.jittered_net()
    gu.log("[full] jittered net 400x400x50 / 1400 strands, FP32-split graph")
    case, res, diag = run_graph(gu, ctx, wl, alp.PREC_FP32_SPLIT, replays=1)
    del case
    torch.cuda.empty_cache()
    out = sampled_check(gu, wl, res, diag, alp.PREC_FP32_SPLIT, n_beam_sample=6, n_cells_sample=40,
                        seed=9, region=(np.array([0.9, 0.9, 0.0]), np.array([0.92, 0.92, 0.25])))
    gu.log(f"[full]   {out}")
    # another storage order of the same cells: identical sources and weights
    perm = np.random.default_rng(4005).permutation(wl["C"].shape[0])
    wl2 = dict(wl)
    wl2["C"], wl2["V"], wl2["U"] = wl["C"][perm], wl["V"][perm], wl["U"][perm]
    case2, res2, diag2 = run_graph(gu, ctx, wl2, alp.PREC_FP32_SPLIT, replays=0)
    del case2
    assert np.array_equal(res2["S"], res["S"][perm])
    assert np.array_equal(res2["w"], res["w"])
    assert np.array_equal(res2["f"], res["f"])
    assert diag2["cons_rel_err"] <= 1e-12


def test_batched_scenarios_full_size_sampled(gu, ctx):
    """64 independent cases (0.5M-4M cells each, 1-500 stems of 20-300 CVs,
    eps/h 1-3 per stem) in one graph-captured step; sampled parity on three
    cases, exact conservation on all of them."""
    from oracle import oracle
    n_cases = 64
    wls = [W.scenario(c) for c in range(n_cases)]
    gu.log(f"[full] batched scenarios: {n_cases} cases, "
           f"{sum(w['C'].shape[0] for w in wls)} cells, {sum(w['beams']['P'].shape[0] for w in wls)} points")
    cases = [gu.GpuCase(ctx, wl, alp.PREC_FP32_SPLIT) for wl in wls]
    flags = alp.USE_GRAPH
    gu.step_batched(ctx, cases, flags)
    gu.step_batched(ctx, cases, flags)
    diags = [ctx.diag(i) for i in range(n_cases)]
    alp.alp_invalidate(ctx.h)
    for i, d in enumerate(diags):
        assert d["n_overflow"] == 0 and d["n_invalid"] == 0, (i, d)
        if d["n_zero_weight"] == 0:
            assert d["cons_rel_err"] <= 1e-12, (i, d)
    rng = np.random.default_rng(77)
    for i in sorted(rng.choice(n_cases, size=3, replace=False).tolist()):
        wl = wls[i]
        res = cases[i].results()
        gu.log(f"[full]   case {i}: {wl['C'].shape[0]} cells, {len(wl['beams']['offsets']) - 1} stems")
        out = sampled_check(gu, wl, res, diags[i], alp.PREC_FP32_SPLIT, n_beam_sample=5,
                            n_cells_sample=60, seed=100 + i)
        gu.log(f"[full]   {out}")


def test_canopy_integrated_full_size_sampled(gu, ctx):
    """The bench canopy under the segment-integrated rule, FP32-split graph
    step: sampled parity (each output depends only on the beams that reach it,
    as under the nearest rule) and the exact balance."""
    wl = W.canopy(n=256, n_stems=2000)
    wl["params"] = dict(wl["params"], proj_mode="integrated")
    gu.log("[full] canopy 256^3 / 2000 stems, integrated rule, FP32-split graph")
    case, res, diag = run_graph(gu, ctx, wl, alp.PREC_FP32_SPLIT, replays=1)
    del case
    torch.cuda.empty_cache()
    gu.log(f"[full]   (cell, segment) pairs {diag['n_pairs']}, band cells {diag['n_band_cells']}")
    out = sampled_check(gu, wl, res, diag, alp.PREC_FP32_SPLIT, n_beam_sample=8, n_cells_sample=80,
                        seed=15)
    gu.log(f"[full]   {out}")
