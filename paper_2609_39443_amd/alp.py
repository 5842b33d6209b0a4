"""Thin ctypes binding of libalp (include/alp.h).

Argument marshalling only: every step of the coupling operator runs in the HIP
kernels of libalp.so.  PyTorch supplies device memory (tensors on ``cuda``,
i.e. HIP) and the stream.  The functions carry the C names; ``Context`` is a
small convenience wrapper around them.  Importing this module does not need a
GPU; loading the library does need libalp.so, and using it needs a GPU.
"""
from __future__ import annotations

import ctypes as ct
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libalp.so")

ALP_OK = 0
STATUS = {0: "ALP_OK", -1: "ALP_ERR_INVALID_ARG", -2: "ALP_ERR_HIP", -3: "ALP_ERR_OOM",
          -4: "ALP_ERR_CAPTURE", -5: "ALP_ERR_SHAPE", -6: "ALP_ERR_CAPACITY"}
PREC_FP64, PREC_FP32_SPLIT = 0, 1
DRAG_FULLMAG, DRAG_COMPONENTWISE = 0, 1
SAMPLE_CELL, SAMPLE_KERNEL = 0, 1
PROJ_NEAREST, PROJ_INTEGRATED = 0, 1
USE_GRAPH, CHECKED, AUTOTUNE = 1, 2, 4

# every symbol include/alp.h declares
EXPORTS = ("alp_create", "alp_destroy", "alp_last_error", "alp_bin_cells", "alp_mesh_destroy",
           "alp_sample", "alp_drag", "alp_spread", "alp_step_batched", "alp_get_diag",
           "alp_invalidate", "alp_version", "alp_step_profile", "alp_stage_name", "alp_autotune",
           "alp_beam_geometry", "alp_step_noalloc", "alp_get_tuning", "alp_set_tuning",
           "alp_autotune_binning")


class AlpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class alp_beams(ct.Structure):
    _fields_ = [("n_beams", ct.c_int32), ("reserved0", ct.c_int32), ("n_points", ct.c_int64),
                ("offsets", ct.c_void_p), ("P", ct.c_void_p), ("P_spread", ct.c_void_p),
                ("e_t", ct.c_void_p), ("Pdot", ct.c_void_p), ("d", ct.c_void_p), ("L", ct.c_void_p),
                ("eps", ct.c_void_p), ("Cdn", ct.c_void_p), ("Cdt", ct.c_void_p), ("ls", ct.c_void_p),
                ("n_p", ct.c_void_p), ("e_up", ct.c_void_p), ("A", ct.c_void_p), ("CMn", ct.c_void_p),
                ("CMt", ct.c_void_p), ("a_b", ct.c_void_p)]


class alp_params(ct.Structure):
    _fields_ = [("rho", ct.c_double), ("alpha_f", ct.c_double), ("tau", ct.c_double),
                ("prec", ct.c_int32), ("drag_form", ct.c_int32), ("sample_mode", ct.c_int32),
                ("proj_mode", ct.c_int32)]


class alp_diag(ct.Structure):
    _fields_ = [("n_outside", ct.c_int64), ("n_fallback", ct.c_int64),
                ("n_fallback_degenerate", ct.c_int64), ("n_zero_weight", ct.c_int64),
                ("n_band_cells", ct.c_int64), ("n_pairs", ct.c_int64), ("n_overflow", ct.c_int64),
                ("n_invalid", ct.c_int64), ("F_beam", ct.c_double * 3), ("F_fluid", ct.c_double * 3),
                ("cons_rel_err", ct.c_double), ("n_sample_empty", ct.c_int64),
                ("n_guard_fp64", ct.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("F_beam", "F_fluid")}
        d["F_beam"] = list(self.F_beam)
        d["F_fluid"] = list(self.F_fluid)
        return d


class alp_case(ct.Structure):
    _fields_ = [("mesh", ct.c_void_p), ("U", ct.c_void_p), ("beams", alp_beams),
                ("params", alp_params), ("f_prev", ct.c_void_p), ("f", ct.c_void_p),
                ("S", ct.c_void_p), ("U_s", ct.c_void_p), ("w", ct.c_void_p), ("P_s", ct.c_void_p),
                ("cell_a", ct.c_void_p), ("cell_s", ct.c_void_p), ("dUdt", ct.c_void_p)]


class alp_tuning(ct.Structure):
    _fields_ = [("sample_lanes", ct.c_int32), ("sample_waves", ct.c_int32), ("weights_grab", ct.c_int32),
                ("weights_waves", ct.c_int32), ("spread_waves", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class alp_beam_state(ct.Structure):
    _fields_ = [("n_beams", ct.c_int32), ("reserved0", ct.c_int32), ("n_points", ct.c_int64),
                ("offsets", ct.c_void_p), ("Cb", ct.c_void_p), ("Wref", ct.c_void_p), ("W", ct.c_void_p),
                ("eps_phys", ct.c_void_p), ("eps_factor", ct.c_double)]


_lib = None


def load():
    """Load libalp.so; raises if it was not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_2609_39443_amd.build")
    lib = ct.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32
    lib.alp_create.argtypes = [ct.c_int, vp, ct.POINTER(vp)]
    lib.alp_destroy.argtypes = [vp]
    lib.alp_last_error.argtypes = [vp]
    lib.alp_last_error.restype = ct.c_char_p
    lib.alp_bin_cells.argtypes = [vp, i64, vp, vp, vp, ct.c_double, i32, ct.POINTER(vp)]
    lib.alp_mesh_destroy.argtypes = [vp]
    lib.alp_sample.argtypes = [vp, vp, vp, ct.POINTER(alp_beams), ct.POINTER(alp_params), vp, vp, vp, vp]
    lib.alp_drag.argtypes = [vp, ct.POINTER(alp_beams), ct.POINTER(alp_params), vp, vp, vp, vp]
    lib.alp_spread.argtypes = [vp, vp, ct.POINTER(alp_beams), ct.POINTER(alp_params), vp, vp, vp, vp]
    lib.alp_step_batched.argtypes = [vp, i32, ct.POINTER(alp_case), u32]
    lib.alp_step_noalloc.argtypes = [vp, i32, ct.POINTER(alp_case)]
    lib.alp_get_diag.argtypes = [vp, i32, ct.POINTER(alp_diag)]
    lib.alp_invalidate.argtypes = [vp]
    lib.alp_version.restype = ct.c_char_p
    lib.alp_step_profile.argtypes = [vp, i32, ct.POINTER(alp_case), ct.POINTER(ct.c_double), i32,
                                     ct.POINTER(i32)]
    lib.alp_step_profile.restype = ct.c_int
    lib.alp_autotune.argtypes = [vp, i64, vp, vp, vp, i32, ct.POINTER(alp_case), i32, u32, i32,
                                 ct.POINTER(ct.c_double), ct.POINTER(i32), ct.POINTER(ct.c_double)]
    lib.alp_autotune.restype = ct.c_int
    lib.alp_get_tuning.argtypes = [vp, ct.POINTER(alp_tuning)]
    lib.alp_set_tuning.argtypes = [vp, ct.POINTER(alp_tuning)]
    lib.alp_autotune_binning.argtypes = [vp, i32, ct.POINTER(alp_case), ct.POINTER(vp), ct.POINTER(vp),
                                         ct.POINTER(vp), u32, i32, ct.POINTER(ct.c_double), ct.POINTER(i32),
                                         ct.POINTER(ct.c_double)]
    lib.alp_beam_geometry.argtypes = [vp, vp, ct.POINTER(alp_beam_state), vp, vp, vp, vp]
    lib.alp_beam_geometry.restype = ct.c_int
    lib.alp_stage_name.argtypes = [i32]
    lib.alp_stage_name.restype = ct.c_char_p
    for name in ("alp_create", "alp_destroy", "alp_bin_cells", "alp_mesh_destroy", "alp_sample",
                 "alp_drag", "alp_spread", "alp_step_batched", "alp_get_diag", "alp_invalidate",
                 "alp_step_noalloc", "alp_get_tuning", "alp_set_tuning", "alp_autotune_binning"):
        getattr(lib, name).restype = ct.c_int
    _lib = lib
    return lib


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libalp takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libalp takes contiguous tensors")
    return t.data_ptr()


def _check(ctx_handle, status):
    if status != ALP_OK:
        msg = load().alp_last_error(ctx_handle).decode(errors="replace")
        raise AlpError(status, msg)


# ------------------------------------------------------------ C-named calls --
def alp_create(device=0, stream=None):
    h = ct.c_void_p()
    st = ct.c_void_p(stream) if stream else None
    s = load().alp_create(int(device), st, ct.byref(h))
    if s != ALP_OK:
        raise AlpError(s, "alp_create failed")
    return h


def alp_destroy(ctx):
    _check(None, load().alp_destroy(ctx))


def alp_bin_cells(ctx, C, V, domain_box=None, bin_size=0.0, tile_bins=0):
    h = ct.c_void_p()
    box = None if domain_box is None else (ct.c_double * 6)(*[float(x) for x in domain_box])
    _check(ctx, load().alp_bin_cells(ctx, C.shape[0], _ptr(C), _ptr(V), box, float(bin_size),
                                     int(tile_bins), ct.byref(h)))
    return h


def alp_mesh_destroy(mesh):
    load().alp_mesh_destroy(mesh)


def alp_sample(ctx, mesh, U, beams: alp_beams, params: alp_params, U_s, P_s=None, cell_a=None,
               cell_s=None):
    _check(ctx, load().alp_sample(ctx, mesh, _ptr(U), ct.byref(beams), ct.byref(params), _ptr(U_s),
                                  _ptr(P_s), _ptr(cell_a), _ptr(cell_s)))


def alp_drag(ctx, beams: alp_beams, params: alp_params, U_s, cell_s, f_prev, f):
    _check(ctx, load().alp_drag(ctx, ct.byref(beams), ct.byref(params), _ptr(U_s), _ptr(cell_s),
                                _ptr(f_prev), _ptr(f)))


def alp_spread(ctx, mesh, beams: alp_beams, params: alp_params, f, S, w=None, fhat=None):
    _check(ctx, load().alp_spread(ctx, mesh, ct.byref(beams), ct.byref(params), _ptr(f), _ptr(S),
                                  _ptr(w), _ptr(fhat)))


def alp_step_batched(ctx, cases, flags=0):
    arr = (alp_case * len(cases))(*cases)
    _check(ctx, load().alp_step_batched(ctx, len(cases), arr, int(flags)))


def alp_step_noalloc(ctx, cases):
    arr = (alp_case * len(cases))(*cases)
    _check(ctx, load().alp_step_noalloc(ctx, len(cases), arr))


def alp_get_diag(ctx, case_index=0):
    d = alp_diag()
    _check(ctx, load().alp_get_diag(ctx, int(case_index), ct.byref(d)))
    return d.as_dict()


def alp_invalidate(ctx):
    _check(ctx, load().alp_invalidate(ctx))


def alp_version():
    return load().alp_version().decode()


def alp_step_profile(ctx, cases, max_stages=16):
    arr = (alp_case * len(cases))(*cases)
    ms = (ct.c_double * max_stages)()
    n = ct.c_int32()
    _check(ctx, load().alp_step_profile(ctx, len(cases), arr, ms, max_stages, ct.byref(n)))
    return {load().alp_stage_name(i).decode(): ms[i] for i in range(n.value)}


def alp_autotune(ctx, C, V, cases, tuned_case=0, flags=USE_GRAPH, reps=3, domain_box=None):
    """Pick the binning (bin size, tile edge in bins) that gives the fastest
    step for `cases`; returns {"bin_size", "tile_bins", "ms"}."""
    arr = (alp_case * len(cases))(*cases)
    box = None if domain_box is None else (ct.c_double * 6)(*[float(x) for x in domain_box])
    bs, tb, ms = ct.c_double(), ct.c_int32(), ct.c_double()
    _check(ctx, load().alp_autotune(ctx, C.shape[0], _ptr(C), _ptr(V), box, len(cases), arr,
                                    int(tuned_case), int(flags), int(reps), ct.byref(bs), ct.byref(tb),
                                    ct.byref(ms)))
    return {"bin_size": bs.value, "tile_bins": tb.value, "ms": ms.value}


def alp_get_tuning(ctx):
    t = alp_tuning()
    _check(ctx, load().alp_get_tuning(ctx, ct.byref(t)))
    return t.as_dict()


def alp_set_tuning(ctx, sample_lanes=4, sample_waves=0, weights_grab=4, weights_waves=16, spread_waves=0):
    t = alp_tuning(sample_lanes, sample_waves, weights_grab, weights_waves, spread_waves)
    _check(ctx, load().alp_set_tuning(ctx, ct.byref(t)))


def alp_autotune_binning(ctx, cases, C, V, boxes=None, flags=USE_GRAPH, reps=3):
    """Rebin every case's cells with each candidate (scale of its default bin
    size, tile edge) and keep the fastest; returns {"scale", "tile_bins", "ms",
    "meshes"}: the new meshes (handles the caller destroys with
    alp_mesh_destroy), one per case, in case order."""
    n = len(cases)
    arr = (alp_case * n)(*cases)
    cp = (ct.c_void_p * n)(*[_ptr(c) for c in C])
    vp_ = (ct.c_void_p * n)(*[_ptr(v) for v in V])
    keep = []
    if boxes is None:
        bp = None
    else:
        bx = []
        for b in boxes:
            if b is None:
                bx.append(None)
            else:
                a = (ct.c_double * 6)(*[float(x) for x in b])
                keep.append(a)
                bx.append(ct.cast(a, ct.c_void_p).value)
        bp = (ct.c_void_p * n)(*bx)
    sc, tb, ms = ct.c_double(), ct.c_int32(), ct.c_double()
    _check(ctx, load().alp_autotune_binning(ctx, n, arr, cp, vp_, bp, int(flags), int(reps), ct.byref(sc),
                                            ct.byref(tb), ct.byref(ms)))
    return {"scale": sc.value, "tile_bins": tb.value, "ms": ms.value,
            "meshes": [ct.c_void_p(arr[i].mesh) for i in range(n)]}


def alp_beam_geometry(ctx, mesh, state, P=None, e_t=None, eps=None, counts=None):
    """Actuator points (eq. 15), tangents and local kernel widths of a beam
    state (alp_beam_state with device pointers) into the given device tensors
    (each nullable)."""
    _check(ctx, load().alp_beam_geometry(ctx, mesh, ct.byref(state), _ptr(P), _ptr(e_t), _ptr(eps),
                                         _ptr(counts)))


# ---------------------------------------------------------------- helpers --
class DeviceBeams:
    """Device copy of a beam-set dict (see workloads.py) and its alp_beams view."""

    KEYS3 = ("P", "e_t", "Pdot")

    def __init__(self, beams: dict, device="cuda"):
        import numpy as np
        import torch

        def f64(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)

        self.offsets = torch.as_tensor(np.ascontiguousarray(beams["offsets"], dtype=np.int64), device=device)
        self.t = {k: f64(beams[k]) for k in ("P", "e_t", "Pdot", "d", "L", "eps", "Cdn", "Cdt", "ls",
                                               "n_p", "e_up")}
        for k in ("P_spread", "A", "CMn", "CMt", "a_b"):  # optional
            v = beams.get(k)
            self.t[k] = None if v is None else f64(v)
        self.n_beams = int(self.offsets.shape[0] - 1)
        self.n_points = int(self.t["P"].shape[0])
        self.struct = self.make_struct()

    def make_struct(self):
        t = self.t
        return alp_beams(self.n_beams, 0, self.n_points, _ptr(self.offsets), _ptr(t["P"]),
                         _ptr(t["P_spread"]), _ptr(t["e_t"]), _ptr(t["Pdot"]), _ptr(t["d"]),
                         _ptr(t["L"]), _ptr(t["eps"]), _ptr(t["Cdn"]), _ptr(t["Cdt"]), _ptr(t["ls"]),
                         _ptr(t["n_p"]), _ptr(t["e_up"]), _ptr(t["A"]), _ptr(t["CMn"]), _ptr(t["CMt"]),
                         _ptr(t["a_b"]))


def make_params(params: dict, prec=PREC_FP64):
    form = params.get("drag_form", DRAG_FULLMAG)
    if isinstance(form, str):
        form = {"fullmag": DRAG_FULLMAG, "componentwise": DRAG_COMPONENTWISE}[form]
    mode = params.get("sample_mode", SAMPLE_CELL)
    if isinstance(mode, str):
        mode = {"cell": SAMPLE_CELL, "kernel": SAMPLE_KERNEL}[mode]
    proj = params.get("proj_mode", PROJ_NEAREST)
    if isinstance(proj, str):
        proj = {"nearest": PROJ_NEAREST, "integrated": PROJ_INTEGRATED}[proj]
    return alp_params(float(params["rho"]), float(params.get("alpha_f", 1.0)),
                      float(params.get("tau", 1e-6)), int(prec), int(form), int(mode), int(proj))


class Context:
    """One libalp context on the current torch stream."""

    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.h = alp_create(device, stream)
        self.meshes = []

    def close(self):
        if self.h is not None:
            for m in self.meshes:
                alp_mesh_destroy(m)
            self.meshes = []
            alp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bin_cells(self, C, V, domain_box=None, bin_size=0.0, tile_bins=0):
        m = alp_bin_cells(self.h, C, V, domain_box, bin_size, tile_bins)
        self.meshes.append(m)
        return m

    def diag(self, case_index=0):
        return alp_get_diag(self.h, case_index)
