"""Python wrapper of the plain FP64 CPU oracle (``alp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the product package
``paper_2609_39443_amd`` never does.  The oracle shares no code with the GPU
path; both sides only share the seeded input generators.

The oracle follows Section 3.2 of Taran et al. (arXiv 2609.39443): point
location (eq. 16, 18), upstream sampling (eq. 17), drag (eq. 19 / eq. 6) with
relaxation (eq. 20), nearest-segment projection with the truncated Gaussian
(eq. 21-22), nodal normalisation (Sec. 3.2.4) and the momentum source (eq. 23).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BRUTE, GRID = 0, 1
FULLMAG, COMPONENTWISE = 0, 1
SAMPLE_CELL, SAMPLE_KERNEL = 0, 1
PROJ_NEAREST, PROJ_INTEGRATED = 0, 1
F_OUTSIDE, F_FALLBACK, F_DEGENERATE = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, -O2, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Beams(ct.Structure):
    _fields_ = [("n_beams", ct.c_int32), ("pad_", ct.c_int32), ("n_points", ct.c_int64),
                ("offsets", ct.c_void_p), ("P", ct.c_void_p), ("P_spread", ct.c_void_p),
                ("e_t", ct.c_void_p), ("Pdot", ct.c_void_p), ("d", ct.c_void_p),
                ("L", ct.c_void_p), ("eps", ct.c_void_p), ("Cdn", ct.c_void_p),
                ("Cdt", ct.c_void_p), ("ls", ct.c_void_p), ("n_p", ct.c_void_p),
                ("e_up", ct.c_void_p), ("A", ct.c_void_p), ("CMn", ct.c_void_p),
                ("CMt", ct.c_void_p), ("a_b", ct.c_void_p)]


class _Params(ct.Structure):
    _fields_ = [("rho", ct.c_double), ("alpha_f", ct.c_double), ("tau", ct.c_double),
                ("drag_form", ct.c_int32), ("sample_mode", ct.c_int32), ("proj_mode", ct.c_int32)]


class _Diag(ct.Structure):
    _fields_ = [("n_outside", ct.c_int64), ("n_fallback", ct.c_int64),
                ("n_fallback_degenerate", ct.c_int64), ("n_zero_weight", ct.c_int64),
                ("n_band_cells", ct.c_int64), ("n_pairs", ct.c_int64),
                ("F_beam", ct.c_double * 3), ("F_fluid", ct.c_double * 3),
                ("cons_rel_err", ct.c_double), ("n_sample_empty", ct.c_int64)]

    def as_dict(self) -> dict:
        return {"n_outside": self.n_outside, "n_fallback": self.n_fallback,
                "n_fallback_degenerate": self.n_fallback_degenerate,
                "n_zero_weight": self.n_zero_weight, "n_band_cells": self.n_band_cells,
                "n_pairs": self.n_pairs, "F_beam": np.array(self.F_beam[:]),
                "F_fluid": np.array(self.F_fluid[:]), "cons_rel_err": self.cons_rel_err,
                "n_sample_empty": self.n_sample_empty}


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ct.CDLL(_LIB)
        vp = ct.c_void_p
        lib.orc_mesh_create.argtypes = [ct.c_int64, vp, vp, vp, ct.c_int, ct.POINTER(vp)]
        lib.orc_mesh_destroy.argtypes = [vp]
        lib.orc_mesh_box.argtypes = [vp]
        lib.orc_mesh_box.restype = ct.POINTER(ct.c_double)
        lib.orc_locate_many.argtypes = [vp, ct.c_int64, vp, vp]
        lib.orc_sample.argtypes = [vp, vp, ct.POINTER(_Beams), ct.POINTER(_Params), vp, vp, vp, vp,
                                   vp, ct.POINTER(_Diag), vp, vp]
        lib.orc_drag.argtypes = [ct.POINTER(_Beams), ct.POINTER(_Params), vp, vp, vp, vp, vp]
        lib.orc_spread.argtypes = [vp, ct.POINTER(_Beams), vp, vp, vp, vp, ct.POINTER(_Diag), ct.c_int32]
        lib.orc_seg_weights.argtypes = [vp, vp, vp, ct.c_double, ct.c_double, vp, vp]
        lib.orc_gl_nodes.argtypes = [vp, vp]
        lib.orc_actuator_points.argtypes = [ct.c_int64, vp, vp, vp, vp]
        lib.orc_tangents.argtypes = [ct.c_int32, vp, vp, vp, ct.POINTER(ct.c_int64)]
        lib.orc_local_eps.argtypes = [vp, ct.c_int64, vp, vp, ct.c_double, vp, ct.POINTER(ct.c_int64)]
        lib.orc_step.argtypes = [vp, vp, ct.POINTER(_Beams), ct.POINTER(_Params), vp, vp, vp, vp,
                                 vp, vp, vp, vp, vp, ct.POINTER(_Diag), vp]
        lib.orc_nearest_segment.argtypes = [ct.c_int64, vp, vp, ct.POINTER(ct.c_double),
                                            ct.POINTER(ct.c_double)]
        lib.orc_nearest_segment.restype = ct.c_int64
        _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


class Mesh:
    """Cell centres C [n,3], volumes V [n], optional domain box [lo(3), hi(3)]."""

    def __init__(self, C, V, box=None, mode: int = GRID):
        lib = _load()
        self.C = _f64(C, (-1, 3))
        self.V = _f64(V, (-1,))
        self.n = self.C.shape[0]
        box_a = None if box is None else _f64(box, (6,))
        h = ct.c_void_p()
        rc = lib.orc_mesh_create(self.n, _ptr(self.C), _ptr(self.V), _ptr(box_a), mode, ct.byref(h))
        if rc != 0:
            raise ValueError(f"orc_mesh_create failed ({rc})")
        self._h = h
        self.mode = mode
        self.box = np.array(lib.orc_mesh_box(h)[:6])

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_mesh_destroy(self._h)
            self._h = None

    def locate(self, X):
        X = _f64(X, (-1, 3))
        out = np.empty(X.shape[0], dtype=np.int64)
        rc = _load().orc_locate_many(self._h, X.shape[0], _ptr(X), _ptr(out))
        if rc != 0:
            raise ValueError("orc_locate_many failed")
        return out


class _BeamArgs:
    """Holds contiguous copies of a beam-set dict and the ctypes struct."""

    def __init__(self, beams: dict):
        self.offsets = np.ascontiguousarray(beams["offsets"], dtype=np.int64)
        nb = self.offsets.shape[0] - 1
        self.P = _f64(beams["P"], (-1, 3))
        npnt = self.P.shape[0]
        ps = beams.get("P_spread")
        self.P_spread = None if ps is None else _f64(ps, (-1, 3))
        self.e_t = _f64(beams["e_t"], (-1, 3))
        self.Pdot = _f64(beams["Pdot"], (-1, 3))
        self.d = _f64(beams["d"], (-1,))
        self.L = _f64(beams["L"], (-1,))
        self.eps = _f64(beams["eps"], (-1,))
        self.Cdn = _f64(beams["Cdn"], (-1,))
        self.Cdt = _f64(beams["Cdt"], (-1,))
        self.ls = _f64(beams["ls"], (-1,))
        self.n_p = _f64(beams["n_p"], (-1, 3))
        self.e_up = _f64(beams["e_up"], (-1, 3))
        for name, arr, n in (("e_t", self.e_t, npnt), ("Pdot", self.Pdot, npnt), ("d", self.d, npnt),
                             ("L", self.L, npnt), ("eps", self.eps, npnt), ("Cdn", self.Cdn, nb),
                             ("Cdt", self.Cdt, nb), ("ls", self.ls, nb), ("n_p", self.n_p, nb),
                             ("e_up", self.e_up, nb)):
            if arr.shape[0] != n:
                raise ValueError(f"beams[{name!r}] has {arr.shape[0]} rows, expected {n}")
        # optional Morison inertia inputs (eq. 8)
        opt = lambda k, shape: None if beams.get(k) is None else _f64(beams[k], shape)
        self.A, self.CMn, self.CMt = opt("A", (-1,)), opt("CMn", (-1,)), opt("CMt", (-1,))
        self.a_b = opt("a_b", (-1, 3))
        if self.A is not None and (self.CMn is None or self.CMt is None):
            raise ValueError("beams['A'] needs 'CMn' and 'CMt'")
        self.s = _Beams(nb, 0, npnt, _ptr(self.offsets), _ptr(self.P), _ptr(self.P_spread),
                        _ptr(self.e_t), _ptr(self.Pdot), _ptr(self.d), _ptr(self.L), _ptr(self.eps),
                        _ptr(self.Cdn), _ptr(self.Cdt), _ptr(self.ls), _ptr(self.n_p), _ptr(self.e_up),
                        _ptr(self.A), _ptr(self.CMn), _ptr(self.CMt), _ptr(self.a_b))
        self.n_points = npnt


def _params(params: dict) -> _Params:
    form = params.get("drag_form", FULLMAG)
    if isinstance(form, str):
        form = {"fullmag": FULLMAG, "componentwise": COMPONENTWISE}[form]
    mode = params.get("sample_mode", SAMPLE_CELL)
    if isinstance(mode, str):
        mode = {"cell": SAMPLE_CELL, "kernel": SAMPLE_KERNEL}[mode]
    proj = params.get("proj_mode", PROJ_NEAREST)
    if isinstance(proj, str):
        proj = {"nearest": PROJ_NEAREST, "integrated": PROJ_INTEGRATED}[proj]
    return _Params(float(params["rho"]), float(params.get("alpha_f", 1.0)),
                   float(params.get("tau", 1e-6)), int(form), int(mode), int(proj))


def sample(mesh: Mesh, U, beams: dict, params: dict, dUdt=None) -> dict:
    lib = _load()
    U = _f64(U, (-1, 3))
    A2 = None if dUdt is None else _f64(dUdt, (-1, 3))
    b = _BeamArgs(beams)
    n = b.n_points
    out = {"U_s": np.zeros((n, 3)), "P_s": np.zeros((n, 3)), "cell_a": np.zeros(n, np.int64),
           "cell_s": np.zeros(n, np.int64), "flags": np.zeros(n, np.int32)}
    if A2 is not None:
        out["a_s"] = np.zeros((n, 3))
    d = _Diag()
    rc = lib.orc_sample(mesh._h, _ptr(U), ct.byref(b.s), ct.byref(_params(params)), _ptr(out["U_s"]),
                        _ptr(out["P_s"]), _ptr(out["cell_a"]), _ptr(out["cell_s"]), _ptr(out["flags"]),
                        ct.byref(d), _ptr(A2), _ptr(out.get("a_s")))
    if rc != 0:
        raise ValueError(f"orc_sample failed ({rc})")
    out["diag"] = d.as_dict()
    return out


def drag(beams: dict, params: dict, U_s, cell_s=None, f_prev=None, a_s=None):
    lib = _load()
    b = _BeamArgs(beams)
    U_s = _f64(U_s, (-1, 3))
    cs = None if cell_s is None else np.ascontiguousarray(cell_s, dtype=np.int64)
    fp = None if f_prev is None else _f64(f_prev, (-1, 3))
    A2 = None if a_s is None else _f64(a_s, (-1, 3))
    f = np.zeros((b.n_points, 3))
    rc = lib.orc_drag(ct.byref(b.s), ct.byref(_params(params)), _ptr(U_s), _ptr(cs), _ptr(fp), _ptr(f),
                      _ptr(A2))
    if rc != 0:
        raise ValueError(f"orc_drag failed ({rc})")
    return f


def spread(mesh: Mesh, beams: dict, f, proj_mode=PROJ_NEAREST) -> dict:
    lib = _load()
    if isinstance(proj_mode, str):
        proj_mode = {"nearest": PROJ_NEAREST, "integrated": PROJ_INTEGRATED}[proj_mode]
    b = _BeamArgs(beams)
    f = _f64(f, (-1, 3))
    out = {"S": np.zeros((mesh.n, 3)), "w": np.zeros(b.n_points), "fhat": np.zeros((b.n_points, 3))}
    d = _Diag()
    rc = lib.orc_spread(mesh._h, ct.byref(b.s), _ptr(f), _ptr(out["S"]), _ptr(out["w"]),
                        _ptr(out["fhat"]), ct.byref(d), int(proj_mode))
    if rc != 0:
        raise ValueError(f"orc_spread failed ({rc})")
    out["diag"] = d.as_dict()
    return out


def step(mesh: Mesh, U, beams: dict, params: dict, f_prev=None, dUdt=None) -> dict:
    """One coupling step: sampling, line force, projection (Sec. 3.2)."""
    lib = _load()
    b = _BeamArgs(beams)
    U = _f64(U, (-1, 3))
    A2 = None if dUdt is None else _f64(dUdt, (-1, 3))
    n = b.n_points
    fp = None if f_prev is None else _f64(f_prev, (-1, 3))
    out = {"U_s": np.zeros((n, 3)), "P_s": np.zeros((n, 3)), "cell_a": np.zeros(n, np.int64),
           "cell_s": np.zeros(n, np.int64), "f": np.zeros((n, 3)), "S": np.zeros((mesh.n, 3)),
           "w": np.zeros(n), "fhat": np.zeros((n, 3))}
    d = _Diag()
    rc = lib.orc_step(mesh._h, _ptr(U), ct.byref(b.s), ct.byref(_params(params)), _ptr(fp),
                      _ptr(out["U_s"]), _ptr(out["P_s"]), _ptr(out["cell_a"]), _ptr(out["cell_s"]),
                      _ptr(out["f"]), _ptr(out["S"]), _ptr(out["w"]), _ptr(out["fhat"]), ct.byref(d),
                      _ptr(A2))
    if rc != 0:
        raise ValueError(f"orc_step failed ({rc})")
    out["diag"] = d.as_dict()
    return out


def nearest_segment(X, c):
    """Closest segment of polyline X [n,3] to point c (eq. 21): (index, s, r^2)."""
    X = _f64(X, (-1, 3))
    c = _f64(c, (3,))
    s = ct.c_double()
    r2 = ct.c_double()
    i = _load().orc_nearest_segment(X.shape[0], _ptr(X), _ptr(c), ct.byref(s), ct.byref(r2))
    return int(i), s.value, r2.value


def seg_weights(c, A, B, eps_a, eps_b):
    """Segment-integrated weights (a0, a1) of one (cell, segment) pair (R27),
    and whether the pair is inside the cutoff."""
    c, A, B = (_f64(x, (3,)) for x in (c, A, B))
    a0 = ct.c_double()
    a1 = ct.c_double()
    inside = _load().orc_seg_weights(_ptr(c), _ptr(A), _ptr(B), float(eps_a), float(eps_b),
                                     ct.byref(a0), ct.byref(a1))
    return a0.value, a1.value, bool(inside)


def gl_nodes():
    """The oracle's 8-point Gauss-Legendre nodes and weights on [0, 1]."""
    s = np.zeros(8)
    w = np.zeros(8)
    _load().orc_gl_nodes(_ptr(s), _ptr(w))
    return s, w


def actuator_points(Cb, W, Wref=None):
    """Eq. (15): P_a = C^b + W^ref + W."""
    Cb, W = _f64(Cb, (-1, 3)), _f64(W, (-1, 3))
    Wr = None if Wref is None else _f64(Wref, (-1, 3))
    P = np.zeros_like(Cb)
    if _load().orc_actuator_points(Cb.shape[0], _ptr(Cb), _ptr(Wr), _ptr(W), _ptr(P)) != 0:
        raise ValueError("orc_actuator_points failed")
    return P


def tangents(offsets, X):
    """R28 unit tangents from the current beam-cell centres X; also the number
    of points left with a zero tangent."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    X = _f64(X, (-1, 3))
    e = np.zeros_like(X)
    ndg = ct.c_int64()
    if _load().orc_tangents(len(off) - 1, _ptr(off), _ptr(X), _ptr(e), ct.byref(ndg)) != 0:
        raise ValueError("orc_tangents failed")
    return e, ndg.value


def local_eps(mesh: Mesh, P, eps_phys, factor=2.0):
    """R29 eps_k = max(factor V_c^(1/3), eps_phys_k), c = c(P_k); also the
    number of points outside the domain."""
    P = _f64(P, (-1, 3))
    ep = _f64(eps_phys, (-1,))
    out = np.zeros(P.shape[0])
    nout = ct.c_int64()
    if _load().orc_local_eps(mesh._h, P.shape[0], _ptr(P), _ptr(ep), float(factor), _ptr(out),
                             ct.byref(nout)) != 0:
        raise ValueError("orc_local_eps failed")
    return out, nout.value
