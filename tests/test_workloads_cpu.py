"""The seeded input generators: bitwise reproducible, with the documented
shapes and sizes (the workloads stand in for the paper's cases)."""
import numpy as np
import pytest

from paper_2609_39443_amd import workloads as W


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        if isinstance(a[k], dict):
            _same(a[k], b[k])
        elif isinstance(a[k], np.ndarray):
            assert a[k].dtype == b[k].dtype and np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], k


def _check_beams(b):
    n = b["P"].shape[0]
    nb = len(b["offsets"]) - 1
    assert b["offsets"][0] == 0 and b["offsets"][-1] == n and np.all(np.diff(b["offsets"]) >= 1)
    for k in ("P", "e_t", "Pdot"):
        assert b[k].shape == (n, 3) and b[k].dtype == np.float64
    for k in ("d", "L", "eps"):
        assert b[k].shape == (n,) and np.all(b[k] > 0)
    for k in ("Cdn", "Cdt", "ls"):
        assert b[k].shape == (nb,)
    assert b["n_p"].shape == (nb, 3) and b["e_up"].shape == (nb, 3)
    assert np.allclose(np.linalg.norm(b["e_t"], axis=1), 1.0)


@pytest.mark.parametrize("make", [
    lambda: W.channel(noise=True),
    lambda: W.wave_flume(snapshot=1, nx=60, ny=20, nz=30, n_cv=30),
    lambda: W.canopy(n=32, n_stems=20, cv_range=(5, 20)),
    lambda: W.jittered_net(nx=40, ny=40, nz=10, n_strands=8, n_cv=30, net_lo=0.02, net_hi=0.18,
                           z0=0.03, sag=0.01),
    lambda: W.scenario(3, n_cells_range=(2e4, 5e4), max_beams=6, cv_range=(5, 20)),
])
def test_generators_reproducible_and_well_formed(make):
    a, b = make(), make()
    _same(a, b)
    n = a["C"].shape[0]
    assert a["C"].shape == (n, 3) and a["V"].shape == (n,) and a["U"].shape == (n, 3)
    assert np.all(a["V"] > 0) and np.all(np.isfinite(a["U"]))
    _check_beams(a["beams"])


def test_documented_full_sizes():
    """Sizes quoted for the full workloads (cells and actuator points)."""
    assert W.channel()["C"].shape[0] == 40 * 20 * 20
    assert W.wave_flume()["C"].shape[0] == 1_987_200
    fl = W.wave_flume()
    assert fl["beams"]["P"].shape[0] == 100
    # canopy: 256^3 cells; stems with 20..200 CVs
    can = W.canopy(n=64, n_stems=2000)
    ncv = np.diff(can["beams"]["offsets"])
    assert len(ncv) == 2000 and ncv.min() >= 20 and ncv.max() <= 200
    # the net: 700 x 700 strands of 357 CVs
    net = W.jittered_net(nx=40, ny=40, nz=10)
    assert net["beams"]["P"].shape[0] == 1400 * 357
    # jittered volumes renormalised to the box volume (Sigma V = 2 x 2 x 0.25 m^3 at full size)
    assert np.isclose(net["V"].sum(), (40 * 0.005) * (40 * 0.005) * (10 * 0.005), rtol=1e-12)


def test_flume_stem_uses_the_paper_sampling_distance():
    """The wave-flume stem samples the flow 0.375 m upstream, the offset of the
    paper's flume set-up (tests/golden/paper_constants.json, Sec. 7.4)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    wl = W.wave_flume(snapshot=0, nx=60, ny=20, nz=30, n_cv=30)
    assert np.all(wl["beams"]["ls"] == gold["flume_sampling_distance_m"]["value"])
