"""libalp: MI355X (gfx950) actuator-line coupling operator.

The operator of Taran et al. (arXiv 2609.39443, Sec. 3.2) -- upstream velocity
sampling, quasi-steady Morison drag and a normalised Gaussian projection of the
reaction onto the fluid mesh -- as hand-written HIP kernels behind the C ABI of
include/alp.h.  ``alp`` is the ctypes binding, ``workloads`` builds seeded
synthetic inputs, ``build`` compiles libalp.so.
"""
__all__ = ["alp", "workloads"]
