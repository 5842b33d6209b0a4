"""GPU parity of the point-wise helpers (alp_beam_geometry, through the C ABI)
against the oracle: actuator points of eq. (15) bitwise, tangents and local
kernel widths to the last bits (division, sqrt and cbrt round independently
on the two sides), the counts exactly.  Then the helpers feed a batched step
whose outputs match the oracle's step on the oracle's helper outputs."""
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


def graded_mesh(nx=24, ny=20, nz=30, h=0.01, h0=0.004, q=1.06):
    ze = W.graded_layers(nz, h0, q)
    zc = 0.5 * (ze[:-1] + ze[1:])
    dz = np.diff(ze)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    Z, Y, X = np.meshgrid(zc, y, x, indexing="ij")
    C = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    V = h * h * np.broadcast_to(dz[:, None, None], Z.shape).ravel()
    perm = np.random.default_rng(8).permutation(C.shape[0])
    return C[perm].copy(), V[perm].copy()


def beam_state(seed, n_beams=7):
    """Initial centres, offsets and displacements of beams with uneven
    spacing; beam 1 has a repeated centre, beam 2 is a single point, beam 3
    is all coincident, the last one leaves the domain."""
    rng = np.random.default_rng(seed)
    Cb, Wref, Wd, offs = [], [], [], [0]
    for b in range(n_beams):
        n = {2: 1, 3: 3}.get(b, int(rng.integers(2, 60)))
        start = rng.uniform([0.03, 0.03, 0.005], [0.2, 0.16, 0.02])
        steps = np.abs(rng.normal(size=(n, 3))) * 0.2 + np.array([0, 0, 1.0])
        steps *= rng.uniform(0.3, 1.8, size=(n, 1)) * 0.004
        c = start + np.cumsum(steps, axis=0)
        if b == 1 and n > 4:
            c[3] = c[2]
        if b == 3:
            c[:] = c[0]
        if b == n_beams - 1:
            c[-1] = [-0.1, 0.1, 0.1]
        Cb.append(c)
        Wref.append(1e-4 * rng.normal(size=(n, 3)))
        wd = 0.01 * np.sin(np.linspace(0, 2, n))[:, None] * rng.normal(size=3)
        Wd.append(np.zeros((n, 3)) if b == 3 else wd)  # beam 3 stays coincident
        offs.append(offs[-1] + n)
    return (np.vstack(Cb), np.vstack(Wref), np.vstack(Wd), np.array(offs, dtype=np.int64),
            rng.uniform(0.002, 0.03, size=offs[-1]))


def run_geometry(gu, ctx, mesh, Cb, Wref, Wd, off, eps_phys, factor=2.0):
    dev = gu.dev
    t = {"off": dev(off, torch.int64), "Cb": dev(Cb), "Wref": dev(Wref), "W": dev(Wd), "ep": dev(eps_phys)}
    n = Cb.shape[0]
    st = alp.alp_beam_state(len(off) - 1, 0, n, t["off"].data_ptr(), t["Cb"].data_ptr(), t["Wref"].data_ptr(),
                            t["W"].data_ptr(), t["ep"].data_ptr(), float(factor))
    P = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
    e = torch.zeros_like(P)
    eps = torch.zeros(n, dtype=torch.float64, device="cuda")
    cnt = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    alp.alp_beam_geometry(ctx.h, mesh, st, P, e, eps, cnt)
    torch.cuda.synchronize()
    return gu.host(P), gu.host(e), gu.host(eps), gu.host(cnt)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_beam_geometry_matches_oracle(gu, ctx, seed):
    from oracle import oracle
    C, V = graded_mesh()
    Cb, Wref, Wd, off, ep = beam_state(seed)
    gu.log(f"[helpers] seed {seed}: {len(off) - 1} beams, {Cb.shape[0]} points")
    mesh = ctx.bin_cells(gu.dev(C), gu.dev(V))
    P, e, eps, cnt = run_geometry(gu, ctx, mesh, Cb, Wref, Wd, off, ep)
    Pr = oracle.actuator_points(Cb, Wd, Wref)
    er, ndg = oracle.tangents(off, Cb + Wd)
    om = oracle.Mesh(C, V, None, oracle.GRID)
    epr, nout = oracle.local_eps(om, Pr, ep, 2.0)
    assert np.array_equal(P, Pr)
    assert np.max(np.abs(e - er)) <= 4e-16
    assert np.max(np.abs(eps - epr) / epr) <= 4e-16
    assert int(cnt[0]) == ndg and int(cnt[1]) == nout
    assert ndg >= 4 and nout >= 1  # the single point, the coincident beam, the outside point
    # the local width took over somewhere and the physical one elsewhere
    assert np.any(eps > ep) and np.any(eps == ep)
    # nullable outputs: tangents only
    n = Cb.shape[0]
    e2 = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
    st = alp.alp_beam_state(len(off) - 1, 0, n, gu.dev(off, torch.int64).data_ptr(), 0, 0, 0, 0, 2.0)
    with pytest.raises(RuntimeError):
        alp.alp_beam_geometry(ctx.h, None, st, None, e2, None, None)  # Cb and W are NULL


def test_beam_geometry_rejects_bad_input(gu, ctx):
    Cb, Wref, Wd, off, ep = beam_state(4, n_beams=3)
    n = Cb.shape[0]
    d = {k: gu.dev(v) for k, v in (("Cb", Cb), ("W", Wd), ("ep", ep))}
    bad = off.copy()
    bad[1], bad[2] = bad[2], bad[1]  # decreasing
    for offs, mesh, want_eps in ((bad, None, False), (off, None, True)):
        o = gu.dev(offs, torch.int64)
        st = alp.alp_beam_state(len(offs) - 1, 0, n, o.data_ptr(), d["Cb"].data_ptr(), 0, d["W"].data_ptr(),
                                d["ep"].data_ptr(), 2.0)
        P = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
        eps = torch.zeros(n, dtype=torch.float64, device="cuda") if want_eps else None
        with pytest.raises(RuntimeError):
            alp.alp_beam_geometry(ctx.h, mesh, st, P, None, eps, None)
        assert torch.count_nonzero(P) == 0


def test_helpers_feed_a_step(gu, ctx):
    """Points, tangents and local widths from alp_beam_geometry drive a
    batched step; the oracle runs its own helpers and its own step."""
    from oracle import oracle
    C, V = graded_mesh()
    Cb, Wref, Wd, off, ep = beam_state(5)
    keep = [b for b in range(len(off) - 1) if b not in (2, 3, len(off) - 2)]  # drop zero tangents
    sel = np.concatenate([np.arange(off[b], off[b + 1]) for b in keep])
    Cb, Wref, Wd, ep = Cb[sel], Wref[sel], Wd[sel], ep[sel]
    off = np.concatenate([[0], np.cumsum([off[b + 1] - off[b] for b in keep])]).astype(np.int64)
    mesh = ctx.bin_cells(gu.dev(C), gu.dev(V))
    P, e, eps, cnt = run_geometry(gu, ctx, mesh, Cb, Wref, Wd, off, ep)
    assert int(cnt[0]) == 0
    nb, n = len(off) - 1, Cb.shape[0]
    rng = np.random.default_rng(6)
    U = np.tile([0.25, 0.02, 0.0], (C.shape[0], 1)) + 0.03 * rng.normal(size=C.shape)

    def beams(P_, e_, eps_):
        return W._beamset([P_[off[b]:off[b + 1]] for b in range(nb)], [e_[off[b]:off[b + 1]] for b in range(nb)],
                          [np.zeros((off[b + 1] - off[b], 3)) for b in range(nb)],
                          [np.full(off[b + 1] - off[b], 0.002) for b in range(nb)],
                          [np.full(off[b + 1] - off[b], 0.004) for b in range(nb)],
                          [eps_[off[b]:off[b + 1]] for b in range(nb)], np.full(nb, 1.2), np.full(nb, 0.05),
                          np.full(nb, 0.03), np.zeros((nb, 3)), np.tile([-1.0, 0, 0], (nb, 1)))

    Pr = oracle.actuator_points(Cb, Wd, Wref)
    er, _ = oracle.tangents(off, Cb + Wd)
    epr, _ = oracle.local_eps(oracle.Mesh(C, V, None, oracle.GRID), Pr, ep, 2.0)
    params = {"rho": 1000.0, "tau": 1e-6}
    wl_gpu = {"name": "helpers-gpu", "C": C, "V": V, "U": U, "box": None, "beams": beams(P, e, eps),
              "params": params}
    wl_ref = dict(wl_gpu, beams=beams(Pr, er, epr))
    case = gu.GpuCase(ctx, wl_gpu, alp.PREC_FP64)
    gu.step_batched(ctx, [case])
    res = case.results()
    ref = gu.oracle_step(wl_ref)
    # the inputs differ from the oracle's in the last bits at most (tangents,
    # widths), so the FP64 tolerance of the step applies
    gu.compare(res, ref, ctx.diag(0), ref["diag"], 1e-12, 1e-12, tol_f=1e-12)
