"""The seeded input generators: determinism, sizes and value ranges."""
import numpy as np

import workloads as W


def test_lightcurves_deterministic_and_sized():
    for name, n in (("tiny", 1000), ("large", 3000), ("sqgrid", 3000)):
        a = W.load_lightcurve(name)
        b = W.load_lightcurve(name)
        assert a["t"].size == n and np.array_equal(a["F"], b["F"])
        assert np.all(np.diff(a["t"]) >= 0)
        assert a["tt"].dtype == np.float32
        assert np.all(a["w"] > 0) and np.all(np.isfinite(a["F"]))
        tr = a["truth"]
        assert a["t"].min() >= tr["t0"] - 2 * tr["tE"] and a["t"].max() <= tr["t0"] + 2 * tr["tE"]


def test_batched_lengths_and_truth_ranges():
    trs = W.truths("batched")
    assert len(trs) == 256
    lens = np.array([t["npts"] for t in trs])
    assert lens.min() >= 200 and lens.max() <= 20000
    assert 1500 < np.median(lens) < 2700
    for tr in trs[:8]:
        lc = W.load_lightcurve("batched", trs.index(tr))
        assert lc["t"].size == tr["npts"]
    assert all(0.3 <= t["s"] <= 3 and 1e-4 <= t["q"] <= 0.1 for t in trs)
    assert W.truths("refine")[5] == trs[5]


def test_grids_and_banks():
    u0, al, t0, tE = W.grid_axes("large")
    assert (u0.size, al.size, t0.size, tE.size) == (64, 64, 16, 8)
    assert u0[0] == 1e-3 and abs(u0[-1] - 0.5) < 1e-12
    assert W.map_bank("sqgrid").shape == (384, 2)
    assert W.map_bank("batched").shape == (64, 2)
    p = W.random_trajectories("sqgrid")
    assert p.shape == (100000, 4)
    assert np.array_equal(p, W.random_trajectories("sqgrid"))
