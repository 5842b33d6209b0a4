"""Pins of the oracle's point-wise helpers: the actuator-point reconstruction
of eq. (15), the centreline tangents (the Hermite-spline node derivatives of
Sec. 3.2.2, read as chord-length three-point derivatives) and the local kernel
width eps = max(2 dx_local, eps_phys) proposed in Sec. 8.

The tangents are pinned by geometry: exact on straight lines with any
spacing and on uniformly sampled circles (by symmetry), second-order
convergence on a helix sampled unevenly (a uniform-parameter derivative would
converge at first order there), and reversal.  The local width is pinned by
meshes whose cell sizes are known.
"""
import math

import numpy as np
import pytest

from paper_2609_39443_amd import workloads as W


def test_actuator_points_eq15(oracle_mod):
    rng = np.random.default_rng(1)
    Cb, Wr, Wd = (rng.normal(size=(7, 3)) for _ in range(3))
    P = oracle_mod.actuator_points(Cb, Wd, Wr)
    assert np.array_equal(P, (Cb + Wr) + Wd)
    assert np.array_equal(oracle_mod.actuator_points(Cb, Wd), Cb + Wd)


def test_actuator_points_follow_a_rigid_rotation(oracle_mod):
    """W is a displacement from the initial centre, not a position: a stem
    rotated rigidly about its base by W = R (C - b) + b - C puts every actuator
    point on the rotated stem, at its initial distance from the base, with the
    material offset W^ref rotated along when it is included in the body."""
    rng = np.random.default_rng(4)
    base = np.array([0.3, -0.2, 0.05])
    s = np.sort(rng.uniform(0.0, 0.5, size=9))
    Cb = base + s[:, None] * np.array([0.0, 0.0, 1.0])
    th = 0.4
    R = np.array([[math.cos(th), 0.0, math.sin(th)], [0.0, 1.0, 0.0], [-math.sin(th), 0.0, math.cos(th)]])
    W = (Cb - base) @ R.T + base - Cb
    P = oracle_mod.actuator_points(Cb, W)
    axis = R @ np.array([0.0, 0.0, 1.0])
    assert np.allclose(np.linalg.norm(P - base, axis=1), s, rtol=0, atol=1e-15)
    assert np.allclose(P - base, s[:, None] * axis, rtol=0, atol=1e-15)
    # an offset of 1 cm towards +x on the undeformed stem is carried as a
    # constant vector (the paper's W^ref is fixed): the points shift by it
    off = np.tile([0.01, 0.0, 0.0], (9, 1))
    assert np.allclose(oracle_mod.actuator_points(Cb, W, off) - P, off, rtol=0, atol=1e-15)


def test_actuator_points_sum_left_to_right(oracle_mod):
    """Eq. (15) is summed in its written order, (C^b + W^ref) + W: with
    1 + 2^-53 + 2^-53 the two half-ulp terms each round away, whereas a sum
    that added them first would give 1 + 2^-52.  The GPU path sums in the same
    order, which its bitwise comparisons rely on."""
    h = 2.0 ** -53
    Cb = np.array([[1.0, -1.0, 4.0]])
    Wr = np.array([[h, -h, 4 * h]])
    W = np.array([[h, -h, 4 * h]])
    P = oracle_mod.actuator_points(Cb, W, Wr)
    assert np.array_equal(P, Cb)
    assert not np.array_equal(P, Cb + (Wr + W))


def test_tangents_exact_on_straight_lines(oracle_mod):
    rng = np.random.default_rng(2)
    polys, dirs = [], []
    for n in (2, 3, 5, 40):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t = np.cumsum(rng.uniform(0.1, 3.0, size=n))
        polys.append(rng.normal(size=3) + t[:, None] * d)
        dirs.append(np.tile(d, (n, 1)))
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in polys])])
    X = np.vstack(polys)
    e, ndg = oracle_mod.tangents(off, X)
    assert ndg == 0
    # exact up to the rounding of the chords: u |x| / (shortest step)
    tol = 8 * 2.0 ** -53 * np.abs(X).max() / 0.1
    assert np.max(np.abs(e - np.vstack(dirs))) <= tol


def test_tangents_exact_on_a_uniform_circle(oracle_mod):
    """Interior nodes of a uniformly sampled circle: the tangent is
    perpendicular to the radius and points along the traversal."""
    R, n = 0.7, 24
    th = np.linspace(0.0, 1.5 * math.pi, n)
    X = np.stack([R * np.cos(th), R * np.sin(th), np.full(n, 0.3)], axis=1)
    e, _ = oracle_mod.tangents([0, n], X)
    exact = np.stack([-np.sin(th), np.cos(th), np.zeros(n)], axis=1)
    assert np.max(np.abs(e[1:-1] - exact[1:-1])) <= 1e-15
    # the ends are one-sided: second order, not exact
    assert 1e-6 < np.max(np.abs(e[[0, -1]] - exact[[0, -1]])) < 0.02


def _helix_error(oracle_mod, n):
    # parameter steps alternating 1 : 3, a pattern that halving the spacing keeps
    steps = np.where(np.arange(n - 1) % 2 == 0, 0.5, 1.5)
    s = np.concatenate([[0.0], np.cumsum(steps)])
    s *= 4.0 * math.pi / s[-1]
    a, c = 0.3, 0.1
    X = np.stack([a * np.cos(s), a * np.sin(s), c * s], axis=1)
    d = np.stack([-a * np.sin(s), a * np.cos(s), np.full(n, c)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e, ndg = oracle_mod.tangents([0, n], X)
    assert ndg == 0
    err = np.linalg.norm(e - d, axis=1)
    return err[1:-1].max(), err[[0, -1]].max()


def test_tangents_second_order_on_an_uneven_helix(oracle_mod):
    """Halving the spacing (steps alternating 1 : 3) divides the tangent error
    by about four, inside and at the ends.  A derivative taken with a uniform
    parameter would converge at first order on this spacing."""
    errs = [_helix_error(oracle_mod, n) for n in (101, 201, 401)]
    for (i0, e0), (i1, e1) in zip(errs[:-1], errs[1:]):
        assert 3.5 < i0 / i1 < 4.5, errs
        assert 3.5 < e0 / e1 < 4.5, errs


def test_tangents_reverse_with_the_beam_and_handle_degenerate_nodes(oracle_mod):
    rng = np.random.default_rng(4)
    X = np.cumsum(rng.normal(size=(9, 3)), axis=0)
    e, _ = oracle_mod.tangents([0, 9], X)
    er, _ = oracle_mod.tangents([0, 9], X[::-1])
    assert np.max(np.abs(er[::-1] + e)) <= 1e-15
    # a repeated centre falls back to the neighbouring chord; a single centre
    # and an all-coincident beam give zero tangents, counted
    Y = np.array([[0.0, 0, 0], [0, 0, 1], [0, 0, 1], [0, 1, 1], [5, 5, 5], [1, 1, 1], [1, 1, 1]])
    e, ndg = oracle_mod.tangents([0, 4, 5, 7], Y)
    assert ndg == 3
    assert np.allclose(e[0], [0, 0, 1]) and np.allclose(e[1], [0, 0, 1])
    assert np.allclose(e[2], [0, 1, 0]) and np.allclose(e[3], [0, 1, 0])
    assert np.all(e[4:] == 0)


def test_local_eps_on_uniform_and_graded_meshes(oracle_mod):
    h = 0.01
    C, V = W.uniform_mesh(10, 10, 10, h)
    m = oracle_mod.Mesh(C, V, None, 1)
    rng = np.random.default_rng(5)
    P = rng.uniform(0.005, 0.095, size=(50, 3))
    ep = rng.uniform(0.5, 3.0, size=50) * h
    eps, nout = oracle_mod.local_eps(m, P, ep)
    assert nout == 0
    assert np.allclose(eps, np.maximum(2 * h, ep), rtol=2e-16, atol=0)
    # a factor of 1 and a physical width below the cell size
    eps1, _ = oracle_mod.local_eps(m, P, np.full(50, 0.1 * h), factor=1.0)
    assert np.allclose(eps1, h, rtol=2e-16, atol=0)
    # two blocks of different cell size: each point takes its own block's size
    C2, V2 = W.uniform_mesh(4, 4, 4, 0.04, origin=(0.1, 0.0, 0.0))
    mg = oracle_mod.Mesh(np.vstack([C, C2]), np.concatenate([V, V2]), None, 1)
    Q = np.array([[0.05, 0.05, 0.05], [0.17, 0.07, 0.09], [0.5, 0.5, 0.5]])
    eg, nout = oracle_mod.local_eps(mg, Q, np.full(3, 0.001))
    assert nout == 1
    assert eg[0] == pytest.approx(0.02, rel=2e-16) and eg[1] == pytest.approx(0.08, rel=2e-16)
    assert eg[2] == 0.001
