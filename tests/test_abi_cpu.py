"""CPU checks of the boundary: libalp.so loads, exports every function that
include/alp.h declares, and the ctypes structs match the C layout (checked by
compiling a small C program against the header with gcc).  No compute calls."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "alp.h")


def declared_functions():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(alp_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("alp_bin_cells", "alp_sample", "alp_drag", "alp_spread", "alp_step_batched"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2609_39443_amd import alp
    lib = alp.load()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(alp.EXPORTS) == set(declared_functions())
    out = subprocess.run(["nm", "-D", "--defined-only", alp.LIB_PATH], capture_output=True, text=True).stdout
    for n in declared_functions():
        assert re.search(rf"\bT {n}\b", out), n
    assert alp.alp_version().startswith("libalp")


def test_struct_layout_matches_header(tmp_path):
    from paper_2609_39443_amd import alp
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "alp.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(alp_beams), '
                    'sizeof(alp_params), sizeof(alp_diag), sizeof(alp_case), offsetof(alp_case, beams), '
                    'offsetof(alp_case, params), offsetof(alp_diag, F_beam), sizeof(alp_beam_state), '
                    'offsetof(alp_beam_state, eps_factor), sizeof(alp_tuning));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ct.sizeof(alp.alp_beams), ct.sizeof(alp.alp_params), ct.sizeof(alp.alp_diag),
            ct.sizeof(alp.alp_case), alp.alp_case.beams.offset, alp.alp_case.params.offset,
            alp.alp_diag.F_beam.offset, ct.sizeof(alp.alp_beam_state), alp.alp_beam_state.eps_factor.offset,
            ct.sizeof(alp.alp_tuning)]
    assert got == want


def test_null_context_is_rejected_without_gpu():
    from paper_2609_39443_amd import alp
    lib = alp.load()
    assert lib.alp_destroy(None) == -1
    assert lib.alp_invalidate(None) == -1


def test_device_gauss_legendre_table_is_the_8_point_rule():
    """The tabulated abscissae and weights the device uses for short segments
    of the integrated rule are those of 8-point Gauss-Legendre quadrature."""
    src = open(os.path.join(ROOT, "paper_2609_39443_amd", "csrc", "alp_internal.h")).read()
    tab = {}
    for name in ("kX", "kW"):
        m = re.search(r"constexpr double %s\[4\] = \{([^}]*)\}" % name, src)
        assert m, name
        tab[name] = np.array([float(v) for v in m.group(1).split(",")])
    x, w = np.polynomial.legendre.leggauss(8)
    # numpy's own weights carry a few ulps of error
    assert np.allclose(tab["kX"], x[4:], rtol=0, atol=1e-15)
    assert np.allclose(tab["kW"], w[4:], rtol=0, atol=1e-15)
