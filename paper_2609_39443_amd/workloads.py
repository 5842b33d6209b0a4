"""Seeded synthetic inputs for the actuator-line coupling operator.

This module only builds inputs: meshes, velocity fields and beam geometry.  It
contains none of the operator's arithmetic (no point location, sampling, drag,
kernel or normalisation), so both the GPU path and the CPU oracle can use it.
Every generator is bitwise reproducible: NumPy ``Generator(PCG64(seed))`` with
the seeds listed per workload.

The shapes stand in for the paper's workloads (Taran et al., arXiv 2609.39443):
the confined channel of Sec. 5 (kernel width about twice the cell size, 20 beam
CVs, sampling offset about five kernel widths) and the wave-flume stem of
Sec. 7.2-7.4 (stem diameter, drag coefficients, 0.375 m sampling offset projected
onto the vertical plane through the stem).  The canopy, net and batched-scenario
workloads scale these shapes up; no item of any external dataset is used.

A workload is a dict::

    {"name", "C" [n,3] f64, "V" [n] f64, "U" [n,3] f64, "box" (6,) f64 or None,
     "h" (nominal cell size), "beams": {...}, "params": {...}}

``beams`` holds ``offsets`` [B+1] i64 (CSR over points), per point ``P``,
``e_t``, ``Pdot`` [n_p,3], ``d``, ``L``, ``eps`` [n_p], and per beam ``Cdn``,
``Cdt``, ``ls`` [B], ``n_p``, ``e_up`` [B,3].  ``params`` holds ``rho``,
``alpha_f``, ``tau``, ``drag_form``.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_mesh(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)):
    """Uniform Cartesian hex mesh, centres at origin + (i+1/2)h, i fastest."""
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    C = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    V = np.full(C.shape[0], h * h * h)
    return C, V


def _beamset(points, tangents, pdot, d, L, eps, Cdn, Cdt, ls, n_p, e_up):
    offsets = np.zeros(len(points) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in points])
    cat = lambda xs, w: (np.concatenate(xs, axis=0) if xs else np.zeros((0, w) if w else (0,)))
    return {
        "offsets": offsets,
        "P": np.ascontiguousarray(cat(points, 3), dtype=np.float64).reshape(-1, 3),
        "e_t": np.ascontiguousarray(cat(tangents, 3), dtype=np.float64).reshape(-1, 3),
        "Pdot": np.ascontiguousarray(cat(pdot, 3), dtype=np.float64).reshape(-1, 3),
        "d": np.ascontiguousarray(cat(d, 0), dtype=np.float64),
        "L": np.ascontiguousarray(cat(L, 0), dtype=np.float64),
        "eps": np.ascontiguousarray(cat(eps, 0), dtype=np.float64),
        "Cdn": np.asarray(Cdn, dtype=np.float64).reshape(-1),
        "Cdt": np.asarray(Cdt, dtype=np.float64).reshape(-1),
        "ls": np.asarray(ls, dtype=np.float64).reshape(-1),
        "n_p": np.asarray(n_p, dtype=np.float64).reshape(-1, 3),
        "e_up": np.asarray(e_up, dtype=np.float64).reshape(-1, 3),
    }


def _params(rho=1000.0, alpha_f=1.0, tau=1e-6, drag_form=0):
    return {"rho": rho, "alpha_f": alpha_f, "tau": tau, "drag_form": drag_form}


# --------------------------------------------------------------------- C1 --
def channel(noise: bool = True, seed: int = 1001, nx=40, ny=20, nz=20, h=0.01, n_cv=20,
            root=(0.2037, 0.1013, 0.0)):
    """Plain FP64 case: 40x20x20 cells (h = 0.01 m), U = (0.5,0,0) + N(0, 0.05^2),
    one straight vertical cantilever of 20 CVs (d = 2 mm, L = 0.01 m) placed off
    the cell faces; Cdn = 1.2, Cdt = 0, rho = 1000, eps = 2h, l_s = 5 eps."""
    C, V = uniform_mesh(nx, ny, nz, h)
    U = np.zeros_like(C)
    U[:, 0] = 0.5
    if noise:
        U += _rng(seed).normal(0.0, 0.05, size=C.shape)
    L = 0.01
    z = root[2] + (np.arange(n_cv) + 0.5) * L
    P = np.stack([np.full(n_cv, root[0]), np.full(n_cv, root[1]), z], axis=1)
    et = np.tile([0.0, 0.0, 1.0], (n_cv, 1))
    eps = 2.0 * h
    beams = _beamset([P], [et], [np.zeros((n_cv, 3))], [np.full(n_cv, 0.002)], [np.full(n_cv, L)],
                     [np.full(n_cv, eps)], [1.2], [0.0], [5.0 * eps], [[0.0, 0.0, 0.0]],
                     [[-1.0, 0.0, 0.0]])
    return {"name": "channel" + ("" if noise else "-clean"), "C": C, "V": V, "U": U, "box": None,
            "h": h, "beams": beams, "params": _params()}


# --------------------------------------------------------------------- C2 --
def airy_wavenumber(T: float, depth: float, g: float = 9.81) -> float:
    """Linear dispersion omega^2 = g k tanh(k d) solved for k by Newton."""
    w = 2.0 * math.pi / T
    k = w * w / g
    for _ in range(100):
        f = g * k * math.tanh(k * depth) - w * w
        df = g * math.tanh(k * depth) + g * k * depth / math.cosh(k * depth) ** 2
        dk = f / df
        k -= dk
        if abs(dk) < 1e-15 * k:
            break
    return k


def graded_layers(n: int, h0: float, q: float) -> np.ndarray:
    """Layer edges z_0 = 0 < z_1 < ... of a geometric grading h0, h0 q, ..."""
    t = h0 * q ** np.arange(n)
    return np.concatenate([[0.0], np.cumsum(t)])


def wave_flume(snapshot: int = 0, noise: bool = True, nx=300, ny=72, nz=92, hx=0.004, hy=0.004,
               h0=0.002, q=1.015402, n_cv=100, stem_len=0.30, seed_noise=2001, seed_geom=2002):
    """Wave-flume stem: 300 x 72 x 92 cells graded in z (2 mm at the bed to
    about 8 mm, 0.4 m deep), linear Airy orbital field H = 0.1 m, T = 1.5 s,
    depth 0.4 m (crest at the stem, or a quarter period later), one bent stem of
    100 CVs, tip velocity up to 0.2 m/s, eps = 1.5 local cell size."""
    ze = graded_layers(nz, h0, q)
    zc = 0.5 * (ze[:-1] + ze[1:])
    dz = np.diff(ze)
    x = (np.arange(nx) + 0.5) * hx
    y = (np.arange(ny) + 0.5) * hy
    Z, Y, X = np.meshgrid(zc, y, x, indexing="ij")
    C = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    DZ = np.broadcast_to(dz[:, None, None], Z.shape).ravel()
    V = hx * hy * DZ
    depth = float(ze[-1])
    H, T, g = 0.1, 1.5, 9.81
    k = airy_wavenumber(T, depth, g)
    w = 2.0 * math.pi / T
    root = np.array([0.6013, 0.1441, 0.0])
    t0 = k * root[0] / w + snapshot * T / 4.0
    ph = k * C[:, 0] - w * t0
    amp = 0.5 * H * w / math.sinh(k * depth)
    U = np.zeros_like(C)
    U[:, 0] = amp * np.cosh(k * C[:, 2]) * np.cos(ph)
    U[:, 2] = amp * np.sinh(k * C[:, 2]) * np.sin(ph)
    if noise:
        U += _rng(seed_noise).normal(0.0, 0.01, size=C.shape)
    rg = _rng(seed_geom)
    kx = rg.uniform(-0.5, 0.5)
    ky = rg.uniform(-0.1, 0.1)
    L = stem_len / n_cv
    s = (np.arange(n_cv) + 0.5) * L
    P = np.stack([root[0] + 0.5 * kx * s * s, root[1] + 0.5 * ky * s * s, s], axis=1)
    et = np.stack([kx * s, ky * s, np.ones_like(s)], axis=1)
    et /= np.linalg.norm(et, axis=1, keepdims=True)
    pdot = np.zeros_like(P)
    pdot[:, 0] = 0.2 * (s / stem_len) ** 2
    # local cell size at each actuator point, from the mesh definition
    iz = np.clip(np.searchsorted(ze, P[:, 2], side="right") - 1, 0, nz - 1)
    eps = 1.5 * np.cbrt(hx * hy * dz[iz])
    beams = _beamset([P], [et], [pdot], [np.full(n_cv, 0.008)], [np.full(n_cv, L)], [eps],
                     [4.0], [0.01], [0.375], [[0.0, 1.0, 0.0]], [[-1.0, 0.0, 0.0]])
    return {"name": f"wave-flume-s{snapshot}", "C": C, "V": V, "U": U, "box": None, "h": hx,
            "beams": beams, "params": _params(), "k": k}


# --------------------------------------------------------------------- C3 --
def canopy(n=256, h=0.004, n_stems=2000, cv_range=(20, 200), inset=0.05, lean_deg=5.0,
           eps_over_h=2.0, seed_u=3001, seed_geom=3002, noise=True):
    """Canopy batch: n^3 uniform cells (256^3 = 16.8M at h = 4 mm), U = (0.3,0,0)
    + N(0, 0.03^2), 2000 straight stems at random roots on the bed, CV counts
    uniform in 20..200 with L = h, lean up to 5 deg, d in U(1,5) mm, eps = 2h,
    l_s = 5 eps, so neighbouring kernels overlap."""
    C, V = uniform_mesh(n, n, n, h)
    U = np.zeros_like(C)
    U[:, 0] = 0.3
    if noise:
        U += _rng(seed_u).normal(0.0, 0.03, size=C.shape)
    box_len = n * h
    rg = _rng(seed_geom)
    roots = rg.uniform(inset, box_len - inset, size=(n_stems, 2))
    ncv = rg.integers(cv_range[0], cv_range[1] + 1, size=n_stems)
    theta = np.deg2rad(rg.uniform(0.0, lean_deg, size=n_stems))
    phi = rg.uniform(0.0, 2.0 * math.pi, size=n_stems)
    dia = rg.uniform(0.001, 0.005, size=n_stems)
    eps = eps_over_h * h
    pts, tan, pd, dd, LL, ee = [], [], [], [], [], []
    for b in range(n_stems):
        et = np.array([math.sin(theta[b]) * math.cos(phi[b]), math.sin(theta[b]) * math.sin(phi[b]),
                       math.cos(theta[b])])
        s = (np.arange(ncv[b]) + 0.5) * h
        P = np.array([roots[b, 0], roots[b, 1], 0.0])[None, :] + s[:, None] * et[None, :]
        pts.append(P)
        tan.append(np.tile(et, (ncv[b], 1)))
        pd.append(np.zeros((ncv[b], 3)))
        dd.append(np.full(ncv[b], dia[b]))
        LL.append(np.full(ncv[b], h))
        ee.append(np.full(ncv[b], eps))
    B = n_stems
    beams = _beamset(pts, tan, pd, dd, LL, ee, np.full(B, 1.2), np.full(B, 0.01), np.full(B, 5.0 * eps),
                     np.zeros((B, 3)), np.tile([-1.0, 0.0, 0.0], (B, 1)))
    return {"name": f"canopy-{n}^3-{n_stems}", "C": C, "V": V, "U": U, "box": None, "h": h,
            "beams": beams, "params": _params()}


# --------------------------------------------------------------------- C4 --
def fourier_field(X, n_modes=32, amp=0.02, kmin=2 * math.pi / 1.0, kmax=2 * math.pi / 0.05,
                  base=(0.2, 0.0, 0.0), seed=4004):
    """Smooth divergence-free field: base + sum_m A a_m cos(k_m . x + phi_m),
    a_m perpendicular to k_m."""
    rg = _rng(seed)
    U = np.tile(np.asarray(base, dtype=np.float64), (X.shape[0], 1))
    for _ in range(n_modes):
        kd = rg.normal(size=3)
        kd /= np.linalg.norm(kd)
        kmag = rg.uniform(kmin, kmax)
        a = rg.normal(size=3)
        a -= np.dot(a, kd) * kd
        a /= np.linalg.norm(a)
        phs = rg.uniform(0.0, 2.0 * math.pi)
        c = np.cos(X @ (kmag * kd) + phs)
        U += amp * c[:, None] * a[None, :]
    return U


def jittered_net(nx=400, ny=400, nz=50, h=0.005, n_strands=700, n_cv=357, jitter=0.3,
                 sigma_v=0.3, seed_jit=4001, seed_vol=4002, seed_perm=4003, seed_u=4004,
                 net_lo=0.1, net_hi=1.9, z0=0.15, sag=0.05, eps_over_h=2.0):
    """Jittered unstructured mesh and net: 400 x 400 x 50 lattice (h = 5 mm)
    with centres jittered by U(+-0.3h), lognormal volumes (sigma 0.3) rescaled
    to the domain volume, stored in a random order; a 700 x 700-strand square
    net (357 CVs per strand) in sinusoidal sag; velocity = sum of 32 Fourier
    modes."""
    C, _ = uniform_mesh(nx, ny, nz, h)
    C = C + _rng(seed_jit).uniform(-jitter * h, jitter * h, size=C.shape)
    V = h ** 3 * np.exp(sigma_v * _rng(seed_vol).normal(size=C.shape[0]))
    V *= (nx * ny * nz * h ** 3) / V.sum()
    perm = _rng(seed_perm).permutation(C.shape[0])
    C = np.ascontiguousarray(C[perm])
    V = np.ascontiguousarray(V[perm])
    U = fourier_field(C, seed=seed_u)
    span = net_hi - net_lo
    L = span / n_cv
    s = net_lo + (np.arange(n_cv) + 0.5) * L
    lines = net_lo + span * np.arange(n_strands) / max(n_strands - 1, 1)
    eps = eps_over_h * h

    def zf(x, y):
        return z0 - sag * np.sin(np.pi * (x - net_lo) / span) * np.sin(np.pi * (y - net_lo) / span)

    def dzdx(x, y):
        return -sag * (np.pi / span) * np.cos(np.pi * (x - net_lo) / span) * np.sin(np.pi * (y - net_lo) / span)

    def dzdy(x, y):
        return -sag * (np.pi / span) * np.sin(np.pi * (x - net_lo) / span) * np.cos(np.pi * (y - net_lo) / span)

    pts, tan = [], []
    for ym in lines:  # strands along x
        y = np.full(n_cv, ym)
        pts.append(np.stack([s, y, zf(s, y)], axis=1))
        t = np.stack([np.ones(n_cv), np.zeros(n_cv), dzdx(s, y)], axis=1)
        tan.append(t / np.linalg.norm(t, axis=1, keepdims=True))
    for xm in lines:  # strands along y
        x = np.full(n_cv, xm)
        pts.append(np.stack([x, s, zf(x, s)], axis=1))
        t = np.stack([np.zeros(n_cv), np.ones(n_cv), dzdy(x, s)], axis=1)
        tan.append(t / np.linalg.norm(t, axis=1, keepdims=True))
    B = 2 * n_strands
    z3 = [np.zeros((n_cv, 3))] * B
    beams = _beamset(pts, tan, z3, [np.full(n_cv, 0.002)] * B, [np.full(n_cv, L)] * B,
                     [np.full(n_cv, eps)] * B, np.full(B, 1.2), np.full(B, 0.01), np.full(B, 5.0 * eps),
                     np.zeros((B, 3)), np.tile([-1.0, 0.0, 0.0], (B, 1)))
    return {"name": f"jittered-net-{nx}x{ny}x{nz}-{n_strands}", "C": C, "V": V, "U": U,
            "box": (0.0, 0.0, 0.0, nx * h, ny * h, nz * h), "h": h, "beams": beams,
            "params": _params(), "perm": perm}


# --------------------------------------------------------------------- C5 --
def scenario(case: int, n_cells_range=(0.5e6, 4.0e6), max_beams=500, cv_range=(20, 300),
             h=0.004, base_seed=5000):
    """One of the batched scenarios: a 2n x n x n uniform mesh (N log-uniform in
    0.5M..4M), U0 in U(0.1, 0.5) with 10 % noise, 1..500 stems of 20..300 CVs,
    eps/h in U(1,3) per stem, Cdn in U(1,4), lean up to 10 deg."""
    rg = _rng(base_seed + case)
    N = math.exp(rg.uniform(math.log(n_cells_range[0]), math.log(n_cells_range[1])))
    n = max(4, int(round((N / 2.0) ** (1.0 / 3.0))))
    C, V = uniform_mesh(2 * n, n, n, h)
    U0 = rg.uniform(0.1, 0.5)
    U = np.zeros_like(C)
    U[:, 0] = U0
    U += rg.normal(0.0, 0.1 * U0, size=C.shape)
    B = int(rg.integers(1, max_beams + 1))
    pts, tan, pd, dd, LL, ee = [], [], [], [], [], []
    Cdn = rg.uniform(1.0, 4.0, size=B)
    eoh = rg.uniform(1.0, 3.0, size=B)
    ls = 5.0 * eoh * h
    for b in range(B):
        ncv = int(rg.integers(cv_range[0], cv_range[1] + 1))
        Lb = 0.8 * n * h / ncv
        inset = ls[b] + 3.0 * eoh[b] * h
        lo, hx_, hy_ = inset, 2 * n * h - inset, n * h - inset
        rx = rg.uniform(lo, max(lo, hx_))
        ry = rg.uniform(lo, max(lo, hy_))
        th = math.radians(rg.uniform(0.0, 10.0))
        ph = rg.uniform(0.0, 2.0 * math.pi)
        et = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        s = (np.arange(ncv) + 0.5) * Lb
        pts.append(np.array([rx, ry, 0.0])[None, :] + s[:, None] * et[None, :])
        tan.append(np.tile(et, (ncv, 1)))
        pd.append(rg.normal(0.0, 0.01, size=(ncv, 3)))
        dd.append(np.full(ncv, rg.uniform(0.001, 0.005)))
        LL.append(np.full(ncv, Lb))
        ee.append(np.full(ncv, eoh[b] * h))
    beams = _beamset(pts, tan, pd, dd, LL, ee, Cdn, np.full(B, 0.01), ls, np.zeros((B, 3)),
                     np.tile([-1.0, 0.0, 0.0], (B, 1)))
    return {"name": f"scenario-{case}", "C": C, "V": V, "U": U, "box": None, "h": h,
            "beams": beams, "params": _params()}


def subset_beams(beams: dict, idx) -> dict:
    """Beam set restricted to the beams listed in idx (in that order)."""
    idx = list(idx)
    off = beams["offsets"]
    sl = [np.arange(off[b], off[b + 1]) for b in idx]
    pid = np.concatenate(sl) if sl else np.zeros(0, dtype=np.int64)
    out = {}
    for k in ("P", "e_t", "Pdot", "d", "L", "eps"):
        out[k] = np.ascontiguousarray(beams[k][pid])
    if beams.get("P_spread") is not None:
        out["P_spread"] = np.ascontiguousarray(beams["P_spread"][pid])
    for k in ("Cdn", "Cdt", "ls", "n_p", "e_up"):
        out[k] = np.ascontiguousarray(beams[k][idx])
    o = np.zeros(len(idx) + 1, dtype=np.int64)
    o[1:] = np.cumsum([len(s) for s in sl])
    out["offsets"] = o
    return out
