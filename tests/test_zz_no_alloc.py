"""The allocation-free entry point alp_step_noalloc against alp_step_batched.

alp_step_noalloc runs the same kernels as an uncaptured alp_step_batched,
with its whole per-step workspace in a static device array, so its outputs
must equal the batched step's bitwise (every sum is exact or taken in a fixed
order, independent of where the lists live) and match the oracle to the
tolerances of the parity tests.  Two calls in a row, the second on a smaller
input, check that the contents the array keeps from a call do not leak into
the next; a step whose fixed lists exceed the array is rejected before any
launch and leaves the context usable.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2609_39443_amd import alp  # noqa: E402
from paper_2609_39443_amd import workloads as W  # noqa: E402

TOL = {alp.PREC_FP64: 1e-12, alp.PREC_FP32_SPLIT: 1e-5}


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


def scene(seed, nx, ny, nz, n_beams):
    rng = np.random.default_rng(seed)
    h = 0.01
    C, V = W.uniform_mesh(nx, ny, nz, h)
    pts, tan = [], []
    for _ in range(n_beams):
        n = int(rng.integers(5, 30))
        start = rng.uniform([0.04, 0.04, 0.01], [nx * h - 0.04, ny * h - 0.04, 0.03])
        d0 = np.array([0.0, 0.0, 1.0]) + 0.3 * rng.normal(size=3)
        d0 /= np.linalg.norm(d0)
        P = start + np.cumsum((d0[None, :] + 0.1 * rng.normal(size=(n, 3))) * 0.8 * h, axis=0)
        pts.append(P)
        t = np.gradient(P, axis=0)
        tan.append(t / np.linalg.norm(t, axis=1, keepdims=True))
    k = [p.shape[0] for p in pts]
    beams = W._beamset(pts, tan, [0.02 * rng.normal(size=(m, 3)) for m in k], [np.full(m, 0.003) for m in k],
                       [np.full(m, 0.008) for m in k], [rng.uniform(1.0, 3.0, m) * h for m in k],
                       rng.uniform(1, 3, n_beams), np.full(n_beams, 0.05), rng.uniform(0.02, 0.05, n_beams),
                       np.zeros((n_beams, 3)), np.tile([-1.0, 0, 0], (n_beams, 1)))
    U = np.tile([0.3, 0.0, 0.0], (C.shape[0], 1)) + 0.05 * rng.normal(size=C.shape)
    return {"name": f"noalloc-{seed}", "C": C, "V": V, "U": U, "box": None, "beams": beams,
            "params": {"rho": 1000.0, "alpha_f": 1.0, "tau": 1e-6}}


@pytest.mark.parametrize("prec", [alp.PREC_FP64, alp.PREC_FP32_SPLIT])
def test_noalloc_matches_batched_twice(gu, ctx, prec):
    big = W.canopy(n=48, n_stems=40, cv_range=(5, 40), inset=0.05)
    small = scene(5, 20, 18, 16, 4)
    for wl in (big, small):
        gu.log(f"[noalloc] {wl['name']} prec={prec}: {wl['C'].shape[0]} cells, {wl['beams']['P'].shape[0]} points")
        a = gu.GpuCase(ctx, wl, prec)
        alp.alp_step_noalloc(ctx.h, [a.case_struct()])
        torch.cuda.synchronize()
        ra, da = a.results(), ctx.diag(0)
        b = gu.GpuCase(ctx, wl, prec)
        gu.step_batched(ctx, [b])
        rb, db = b.results(), ctx.diag(0)
        for k in ra:
            assert np.array_equal(ra[k], rb[k]), k
        assert da == db
        ref = gu.oracle_step(wl)
        err = gu.compare(ra, ref, da, ref["diag"], TOL[prec], TOL[prec])
        gu.log(f"[noalloc]   errors {err}")


def test_noalloc_two_cases_and_rejects_oversized(gu, ctx):
    wls = [scene(7, 22, 20, 18, 5), W.channel(noise=True)]
    cases = [gu.GpuCase(ctx, wl, p) for wl, p in zip(wls, (alp.PREC_FP32_SPLIT, alp.PREC_FP64))]
    gu.log("[noalloc] two cases in one call")
    alp.alp_step_noalloc(ctx.h, [c.case_struct() for c in cases])
    torch.cuda.synchronize()
    for i, (wl, c, p) in enumerate(zip(wls, cases, (alp.PREC_FP32_SPLIT, alp.PREC_FP64))):
        ref = gu.oracle_step(wl)
        gu.compare(c.results(), ref, ctx.diag(i), ref["diag"], TOL[p], TOL[p])
    # one bin per tile on a 10^6-cell mesh: the tile lists alone exceed the array
    C, V = W.uniform_mesh(100, 100, 100, 0.01)
    wl = dict(W.channel(noise=False))
    wl["C"], wl["V"] = C, V
    wl["U"] = np.tile([0.5, 0.0, 0.0], (C.shape[0], 1))
    gu.log("[noalloc] oversized: 10^6 cells in one-bin tiles")
    big = gu.GpuCase(ctx, wl, alp.PREC_FP64, tile_bins=1, bin_size=0.005)
    with pytest.raises(alp.AlpError) as err:
        alp.alp_step_noalloc(ctx.h, [big.case_struct()])
    assert err.value.status == -6 and "fixed workspace" in str(err.value)
    alp.alp_step_noalloc(ctx.h, [cases[1].case_struct()])
    ref = gu.oracle_step(wls[1])
    gu.compare(cases[1].results(), ref, ctx.diag(0), ref["diag"], 1e-12, 1e-12)
