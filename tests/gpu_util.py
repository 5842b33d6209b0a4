"""Helpers for the GPU tests: run libalp through its C ABI on numpy workloads
and compare with the FP64 oracle.  Imported by -m gpu tests only (needs torch
with a HIP device and a built libalp.so)."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_2609_39443_amd import alp


def log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


class GpuCase:
    """Device arrays of one workload and the outputs of one step."""

    def __init__(self, ctx: alp.Context, wl: dict, prec=alp.PREC_FP64, tile_bins=0, bin_size=0.0,
                 f_prev=None):
        self.ctx = ctx
        self.wl = wl
        self.C = dev(wl["C"])
        self.V = dev(wl["V"])
        self.U = dev(wl["U"])
        self.mesh = ctx.bin_cells(self.C, self.V, wl.get("box"), bin_size, tile_bins)
        self.beams = alp.DeviceBeams(wl["beams"])
        self.params = alp.make_params(wl["params"], prec)
        n, npnt = self.C.shape[0], self.beams.n_points
        z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")
        self.f = z(npnt, 3)
        self.S = z(n, 3)
        self.U_s = z(npnt, 3)
        self.P_s = z(npnt, 3)
        self.w = z(npnt)
        self.fhat = z(npnt, 3)
        self.cell_a = torch.zeros(npnt, dtype=torch.int64, device="cuda")
        self.cell_s = torch.zeros(npnt, dtype=torch.int64, device="cuda")
        self.f_prev = None if f_prev is None else dev(f_prev)
        self.dUdt = None if wl.get("dUdt") is None else dev(wl["dUdt"])

    def case_struct(self):
        return alp.alp_case(self.mesh, self.U.data_ptr(), self.beams.struct, self.params,
                            None if self.f_prev is None else self.f_prev.data_ptr(),
                            self.f.data_ptr(), self.S.data_ptr(), self.U_s.data_ptr(),
                            self.w.data_ptr(), self.P_s.data_ptr(), self.cell_a.data_ptr(),
                            self.cell_s.data_ptr(), None if self.dUdt is None else self.dUdt.data_ptr())

    def step_unbatched(self):
        h = self.ctx.h
        alp.alp_sample(h, self.mesh, self.U, self.beams.struct, self.params, self.U_s, self.P_s,
                       self.cell_a, self.cell_s)
        alp.alp_drag(h, self.beams.struct, self.params, self.U_s, self.cell_s, self.f_prev, self.f)
        alp.alp_spread(h, self.mesh, self.beams.struct, self.params, self.f, self.S, self.w, self.fhat)
        torch.cuda.synchronize()

    def results(self):
        torch.cuda.synchronize()
        return {k: host(getattr(self, k)) for k in ("f", "S", "U_s", "P_s", "w", "fhat", "cell_a",
                                                     "cell_s")}


def step_batched(ctx: alp.Context, cases, flags=0):
    alp.alp_step_batched(ctx.h, [c.case_struct() for c in cases], flags)
    torch.cuda.synchronize()


def oracle_step(wl, f_prev=None):
    from oracle import oracle
    m = oracle.Mesh(wl["C"], wl["V"], wl.get("box"), oracle.GRID)
    return oracle.step(m, wl["U"], wl["beams"], wl["params"], f_prev=f_prev, dUdt=wl.get("dUdt"))


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    den = np.max(np.linalg.norm(b, axis=1)) if b.size else 0.0
    num = np.max(np.linalg.norm(a - b, axis=1)) if b.size else 0.0
    return num / den if den > 0 else num


def compare(res, ref, diag, ref_diag, tol_S, tol_w, tol_f=1e-12, check_sample=True, tol_us=0.0):
    """Element-by-element comparison with the oracle; returns a dict of errors."""
    err = {}
    if check_sample:
        assert np.array_equal(res["cell_a"], ref["cell_a"]), "cell_a differs"
        assert np.array_equal(res["cell_s"], ref["cell_s"]), "cell_s differs"
        err["P_s"] = normwise(res["P_s"], ref["P_s"])
        err["U_s"] = normwise(res["U_s"], ref["U_s"])
        # the single-cell sample is a copy; the kernel-weighted one (R25) is a
        # sum whose order differs from the oracle's
        assert err["P_s"] <= 1e-15 and err["U_s"] <= tol_us, err
    err["f"] = normwise(res["f"], ref["f"])
    assert err["f"] <= tol_f, err
    zw = ref["w"] == 0
    assert np.all(res["w"][zw] == 0), "weight on a node that catches no cell"
    err["w"] = float(np.max(np.abs(res["w"][~zw] - ref["w"][~zw]) / ref["w"][~zw])) if np.any(~zw) else 0.0
    assert err["w"] <= tol_w, err
    err["S"] = normwise(res["S"], ref["S"])
    assert err["S"] <= tol_S, err
    # cells outside the band are exactly zero on both sides
    zero_ref = np.all(ref["S"] == 0, axis=1)
    assert np.all(res["S"][zero_ref] == 0), "non-zero source outside the band"
    err["cons"] = diag["cons_rel_err"]
    if ref_diag["n_zero_weight"] == 0:
        assert diag["cons_rel_err"] <= 1e-12, diag
    else:
        # dropped nodes (w_k = 0): the error is exactly their share of the load
        assert abs(diag["cons_rel_err"] - ref_diag["cons_rel_err"]) <= 1e-12 * max(1.0, ref_diag["cons_rel_err"]), (diag, ref_diag)
    for a in range(3):
        scale = max(1e-300, float(np.max(np.abs(ref_diag["F_beam"]))))
        assert abs(diag["F_beam"][a] - ref_diag["F_beam"][a]) <= 1e-12 * scale, (diag, ref_diag)
        assert abs(diag["F_fluid"][a] - ref_diag["F_fluid"][a]) <= 1e-12 * scale, (diag, ref_diag)
    for k in ("n_outside", "n_fallback", "n_fallback_degenerate", "n_zero_weight", "n_pairs",
              "n_band_cells", "n_sample_empty"):
        if check_sample or k not in ("n_outside", "n_fallback", "n_fallback_degenerate", "n_sample_empty"):
            assert diag[k] == ref_diag[k], (k, diag[k], ref_diag[k])
    assert diag["n_overflow"] == 0 and diag["n_invalid"] == 0, diag
    return err
