"""Pins of the oracle's segment-integrated projection (the 3D Gaussian
integrated along each segment and summed over every segment within the
cutoff, the projection change proposed in the paper's conclusions).

Each pin checks it against something other than its own closed form:
adaptive quadrature of the defining integral in 3D, the Gauss-Legendre rule
of numpy, the 2D kernel of eq. (22) that the sum must reach along a straight
line (with the axial mass and first moment of the included span, which fix
the split between the two nodes of a segment), the exact balance of
Sec. 3.2.4, the point kernel for single-CV beams, continuity across the seam
of the nearest-segment rule, and invariances.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from test_oracle_pins import _random_scene, beams_of, params


def _g3(x, eps):
    return math.exp(-float(x @ x) / eps ** 2) / (math.pi ** 1.5 * eps ** 3)


def _weights_by_quadrature(c, A, B, eps):
    """a0, a1 from the definition: int_0^1 (1-s | s) g(c - A - s (B - A)) l ds."""
    c, A, B = (np.asarray(v, float) for v in (c, A, B))
    e = B - A
    l = float(np.linalg.norm(e))
    f0 = lambda s: (1.0 - s) * _g3(c - A - s * e, eps) * l
    f1 = lambda s: s * _g3(c - A - s * e, eps) * l
    # split the interval at the foot of the perpendicular (the integrand's peak)
    s_f = float(np.clip((c - A) @ e / (e @ e), 0.0, 1.0))
    pts = [s_f] if 0.0 < s_f < 1.0 else None
    kw = dict(epsabs=0.0, epsrel=1e-13, limit=400, points=pts)
    return quad(f0, 0.0, 1.0, **kw)[0], quad(f1, 0.0, 1.0, **kw)[0]


def test_gl_nodes_are_gauss_legendre(oracle_mod):
    s, w = oracle_mod.gl_nodes()
    x, wx = np.polynomial.legendre.leggauss(8)
    o = np.argsort(s)
    assert np.allclose(s[o], (x + 1.0) / 2.0, rtol=0, atol=1e-15)
    assert np.allclose(w[o], wx / 2.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lam", [1e-7, 1e-3, 0.05, 0.1249, 0.1251, 0.4, 1.0, 3.0, 12.0, 60.0])
def test_seg_weights_match_adaptive_quadrature(oracle_mod, lam):
    """Both branches of the evaluation (quadrature below l = eps/8, closed form
    above) against adaptive quadrature of the 3D integral, at cells all round
    the segment inside the cutoff."""
    rng = np.random.default_rng(int(lam * 1e7) % 2**31)
    eps_a, eps_b = 0.011, 0.009
    eps = 0.5 * (eps_a + eps_b)
    A = np.array([0.1, -0.2, 0.3])
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    B = A + lam * eps * u
    worst, n_in = 0.0, 0
    for _ in range(40):
        # a point within 3 eps of the segment: random axial position (beyond the
        # ends too) and radius
        s = rng.uniform(-0.5, 1.5) if lam > 1e-3 else rng.uniform(-1e3, 1e3)
        r = rng.uniform(0.0, 2.9) * eps
        v = rng.normal(size=3)
        v -= (v @ u) * u
        v /= np.linalg.norm(v)
        c = A + s * lam * eps * u + r * v
        a0, a1, inside = oracle_mod.seg_weights(c, A, B, eps_a, eps_b)
        # the cutoff is the distance to the closed segment
        sf = min(max((c - A) @ (B - A) / ((B - A) @ (B - A)), 0.0), 1.0)
        d = np.linalg.norm(c - A - sf * (B - A))
        assert inside == (d <= 3.0 * eps)
        if not inside:
            assert a0 == 0.0 and a1 == 0.0
            continue
        n_in += 1
        q0, q1 = _weights_by_quadrature(c, A, B, eps)
        scale = q0 + q1
        worst = max(worst, abs(a0 - q0) / scale, abs(a1 - q1) / scale)
    assert n_in >= 10
    assert worst <= 1e-11, worst


def _single_cell(oracle_mod, x):
    return oracle_mod.Mesh(np.asarray([x], float), np.array([1.0]), None, 0)


def test_straight_line_reaches_eq22_with_the_right_moments(oracle_mod):
    """Along a straight line of unequal segments with one eps, the weights of a
    single unit-volume cell sum to the 2D kernel of eq. (22) at its radial
    distance times the axial mass of the included span, and their first moment
    over the node positions is the closed-form first moment of that span."""
    eps = 0.01
    rng = np.random.default_rng(3)
    seg = rng.uniform(0.2, 1.6, size=60) * eps
    z = np.concatenate([[0.0], np.cumsum(seg)])
    P = np.stack([np.zeros_like(z), np.zeros_like(z), z], axis=1)
    b = beams_of([P], eps, L=0.01)
    f = np.zeros((P.shape[0], 3))
    for zc, r in [(0.5 * z[-1] + 0.0031, 0.4 * eps), (0.5 * z[-1] - 0.0123, 1.7 * eps),
                  (0.011, 0.9 * eps), (z[-1] + 0.01, 0.5 * eps)]:
        x = np.array([r, 0.0, zc])
        out = oracle_mod.spread(_single_cell(oracle_mod, x), b, f, proj_mode="integrated")
        w = out["w"]
        # segments within 3 eps of the cell (distance to the closed segment)
        lo, hi = None, None
        for i in range(len(seg)):
            dz = max(z[i] - zc, 0.0, zc - z[i + 1])
            if r * r + dz * dz <= 9 * eps * eps:
                lo = z[i] if lo is None else lo
                hi = z[i + 1]
        a, bb = (lo - zc) / eps, (hi - zc) / eps
        eta = math.exp(-(r / eps) ** 2) / (math.pi * eps ** 2)
        mass = 0.5 * (math.erf(bb) - math.erf(a))
        assert w.sum() == pytest.approx(eta * mass, rel=1e-13)
        # first moment: int (zc + eps x) e^{-x^2} eps dx over [a, b] / (sqrt(pi) eps)
        m1 = zc * mass + eps * (math.exp(-a * a) - math.exp(-bb * bb)) / (2.0 * math.sqrt(math.pi))
        assert (w * z).sum() == pytest.approx(eta * m1, rel=1e-12)
        assert out["diag"]["n_pairs"] == int(np.count_nonzero(
            [r * r + max(z[i] - zc, 0.0, zc - z[i + 1]) ** 2 <= 9 * eps * eps for i in range(len(seg))]))
    # deep inside the line the span covers the whole kernel: eq. (22) to 1e-4
    x = np.array([0.8 * eps, 0.0, 0.5 * z[-1]])
    w = oracle_mod.spread(_single_cell(oracle_mod, x), b, f, proj_mode="integrated")["w"]
    eta = math.exp(-0.64) / (math.pi * eps ** 2)
    assert abs(w.sum() / eta - 1.0) < 1.2e-4


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_integrated_conserves_force_on_random_scenes(oracle_mod, seed):
    """Sec. 3.2.4 holds for any weights: sum_j S_j V_j = -sum_k f_k L_k."""
    C, V, U, b = _random_scene(seed)
    m = oracle_mod.Mesh(C, V, None, 1)
    near = oracle_mod.step(m, U, b, params())
    r = oracle_mod.step(m, U, b, params(proj_mode="integrated"))
    assert r["diag"]["n_zero_weight"] == 0
    assert r["diag"]["cons_rel_err"] <= 1e-14
    assert r["diag"]["n_pairs"] > near["diag"]["n_pairs"]
    # the sampled velocities and line forces do not depend on the projection
    assert np.array_equal(r["f"], near["f"])
    # both modes put the same load into the fluid
    assert np.allclose(r["diag"]["F_fluid"], near["diag"]["F_fluid"], rtol=1e-13, atol=1e-18)


def test_single_cv_beams_keep_the_point_kernel(oracle_mod):
    C, V, U, b = _random_scene(5, n_beams=6)
    single = beams_of([b["P"][b["offsets"][i]:b["offsets"][i] + 1] for i in range(6)], 0.02, L=0.01)
    m = oracle_mod.Mesh(C, V, None, 1)
    f = np.tile([0.2, -0.1, 0.05], (6, 1))
    a = oracle_mod.spread(m, single, f, proj_mode="nearest")
    c = oracle_mod.spread(m, single, f, proj_mode="integrated")
    assert np.array_equal(a["S"], c["S"]) and np.array_equal(a["w"], c["w"])


def _bend_weights(oracle_mod, mode, n_probe):
    """Weights of a unit cell moved along an arc through the inside of a right-
    angle bend, crossing the bisector plane (the seam of the nearest-segment
    rule).  Every probe stays within 3 eps of both segments."""
    eps = 0.01
    P = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.05], [0.05, 0.0, 0.05]])
    b = beams_of([P], eps, L=0.05)
    f = np.zeros((3, 3))
    out = []
    for th in np.linspace(math.pi * 0.15, math.pi * 0.35, n_probe):
        x = np.array([0.0, 0.0, 0.05]) + 1.5 * eps * np.array([math.sin(th), 0.0, -math.cos(th)])
        out.append(oracle_mod.spread(_single_cell(oracle_mod, x), b, f, proj_mode=mode)["w"])
    return np.array(out)


def test_integrated_removes_the_seam(oracle_mod):
    """The integrated weights are continuous in the cell position: halving the
    probe spacing halves the largest jump.  The nearest-segment weights jump
    by a fixed amount at the bisector however fine the probes."""
    jumps = {}
    for mode in ("nearest", "integrated"):
        for n in (41, 81):
            w = _bend_weights(oracle_mod, mode, n)
            jumps[mode, n] = np.max(np.abs(np.diff(w, axis=0)))
    assert jumps["integrated", 81] <= 0.6 * jumps["integrated", 41]
    assert jumps["nearest", 81] >= 0.9 * jumps["nearest", 41]
    assert jumps["nearest", 81] > 10 * jumps["integrated", 81]


def test_zero_length_segment_contributes_nothing(oracle_mod):
    """A repeated point splits one node into two whose weights add up to it;
    every other node keeps its weight."""
    C, V, U, b = _random_scene(7, n_beams=1)
    P = b["P"]
    if P.shape[0] < 4:
        P = np.vstack([P, P[-1] + [0.0, 0.0, 0.01], P[-1] + [0.0, 0.003, 0.02]])
    Pd = np.vstack([P[:3], P[2:]])  # node 2 repeated
    eps = 0.02
    m = oracle_mod.Mesh(C, V, None, 1)
    a = oracle_mod.spread(m, beams_of([P], eps, L=0.01), np.zeros((P.shape[0], 3)), proj_mode="integrated")
    d = oracle_mod.spread(m, beams_of([Pd], eps, L=0.01), np.zeros((Pd.shape[0], 3)), proj_mode="integrated")
    wa, wd = a["w"], d["w"]
    assert np.allclose(wd[:2], wa[:2], rtol=1e-14, atol=0)
    assert wd[2] + wd[3] == pytest.approx(wa[2], rel=1e-14)
    assert np.allclose(wd[4:], wa[3:], rtol=1e-14, atol=0)
    # with a load split between the two halves, the balance stays exact
    fd = np.tile([0.1, 0.2, -0.3], (Pd.shape[0], 1))
    bd = beams_of([Pd], eps, L=0.01)
    r = oracle_mod.spread(m, bd, fd, proj_mode="integrated")
    assert r["diag"]["n_zero_weight"] == 0 and r["diag"]["cons_rel_err"] <= 1e-14


def test_reversal_symmetry(oracle_mod):
    """Reversing a beam's point order reverses its weights and keeps its
    sources."""
    C, V, U, b = _random_scene(11, n_beams=1)
    P = b["P"]
    if P.shape[0] < 3:
        P = np.vstack([P, P[-1] + [0.004, 0.0, 0.01], P[-1] + [0.0, 0.003, 0.02]])
    eps = np.linspace(0.015, 0.025, P.shape[0])
    m = oracle_mod.Mesh(C, V, None, 1)
    f = np.random.default_rng(2).normal(size=P.shape)
    a = oracle_mod.spread(m, beams_of([P], [eps], L=0.01), f, proj_mode="integrated")
    r = oracle_mod.spread(m, beams_of([P[::-1]], [eps[::-1]], L=0.01), f[::-1], proj_mode="integrated")
    assert np.allclose(r["w"][::-1], a["w"], rtol=1e-13, atol=0)
    assert np.max(np.abs(r["S"] - a["S"])) <= 1e-12 * np.max(np.abs(a["S"]))
