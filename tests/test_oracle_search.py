"""Pins of oracle.sampling / oracle.fit / oracle.search (sec. 4.2, Eqs. 5-6)."""
import math

import numpy as np
import pytest

from oracle.fit import fit_and_chi2, neumaier_sum, topk
from oracle.lens import paczynski
from oracle.sampling import (map_geometry32, sample_exact64, sample_mirror32,
                             traj_constants32, trajectory_positions)
from oracle.search import grid_params, search_exact64, search_mirror32

WIN = (0.0, 0.0, 2.0, 2.0, 64, 48)


def _ramp_map(a=0.375, b=-0.25, c=5.0):  # exactly representable in binary32
    j, i = np.mgrid[0:WIN[5], 0:WIN[4]]
    return (a * i + b * j + c).astype(np.float32), (a, b, c)


def test_geometry_closest_approach():
    p = np.array([3.0, 0.2, 15.0, 1.1])
    z = trajectory_positions(p, np.array([3.0, 3.0 + 15.0]))
    assert abs(z[0]) == pytest.approx(0.2, rel=1e-14)
    # direction of motion is (cos a, sin a), perpendicular to the closest-approach vector
    v = z[1] - z[0]
    assert v.real == pytest.approx(math.cos(1.1)) and v.imag == pytest.approx(math.sin(1.1))
    assert (v.conjugate() * z[0]).real == pytest.approx(0.0, abs=1e-14)


def test_samples_at_pixel_centres_are_exact():
    amap = np.random.default_rng(0).uniform(1, 10, (WIN[5], WIN[4])).astype(np.float32)
    # horizontal trajectory along the row of pixel centres j = 20 (alpha = 0)
    dx = WIN[2] / WIN[4]
    y = WIN[1] - WIN[3] / 2 + (20 + 0.5) * WIN[3] / WIN[5]
    x = WIN[0] - WIN[2] / 2 + (np.arange(3, 60) + 0.5) * dx
    # alpha = 0, u0 = y (bx = 0, by = u0), tE = 1, t0 = 0: zeta = (t, u0); t = x
    params = np.array([[0.0, y, 1.0, 0.0]])
    k = traj_constants32(params, 0.0)
    A = sample_mirror32(amap, WIN, k, x.astype(np.float32))
    g = map_geometry32(WIN)
    gx = ((x.astype(np.float32) - g["sx"]) * g["kx"]) + g["ox"]
    on = gx == np.rint(gx)
    assert on.sum() > 10
    assert np.array_equal(A[0][on], amap[20, np.rint(gx[on]).astype(int)])


def test_bilinear_reproduces_linear_ramps():
    amap, (a, b, c) = _ramp_map()
    rng = np.random.default_rng(1)
    params = np.stack([rng.uniform(-1, 1, 20), rng.uniform(0, 0.6, 20), rng.uniform(5, 30, 20),
                       rng.uniform(0, 2 * np.pi, 20)], axis=1)
    t = np.linspace(-25, 25, 400)
    A, P = sample_exact64(amap, WIN, params, t, parts=True)
    on = P["onmap"]
    assert on.sum() > 1000
    g = map_geometry32(WIN)
    gx = (P["zx"] - WIN[0]) * (WIN[4] / WIN[2]) + (WIN[4] / 2 - 0.5)
    gy = (P["zy"] - WIN[1]) * (WIN[5] / WIN[3]) + (WIN[5] / 2 - 0.5)
    assert np.abs(A[on] - (a * gx[on] + b * gy[on] + c)).max() < 1e-12
    A32, P32 = sample_mirror32(amap, WIN, traj_constants32(params, 0.0), t.astype(np.float32),
                               parts=True)
    both = on & P32["onmap"]
    assert both.sum() > 0.99 * on.sum()
    assert np.abs(A32[both] - A[both]).max() < 1e-5  # ramp spans 0..30


def test_off_map_is_paczynski_about_barycentre():
    amap = np.ones((WIN[5], WIN[4]), np.float32)
    params = np.array([[0.0, 1.5, 10.0, 0.3]])  # u0 beyond the window: always off-map
    t = np.linspace(-30, 30, 101)
    A32 = sample_mirror32(amap, WIN, traj_constants32(params, 0.0), t.astype(np.float32))
    z = trajectory_positions(params[0], t)
    assert np.abs(A32[0] / paczynski(np.abs(z)) - 1).max() < 2e-6


def test_profiled_fit_matches_lstsq_and_recovers_noise_free():
    rng = np.random.default_rng(2)
    a = rng.uniform(1, 20, (5, 300))
    F = rng.normal(3, 1, 300)
    w = rng.uniform(0.5, 2.0, 300)
    chi2, Fs, Fb, deg = fit_and_chi2(a, F, w)
    for k in range(5):
        M = np.stack([a[k], np.ones(300)], axis=1) * np.sqrt(w)[:, None]
        sol, res, _, _ = np.linalg.lstsq(M, F * np.sqrt(w), rcond=None)
        assert Fs[k] == pytest.approx(sol[0], rel=1e-11)
        assert Fb[k] == pytest.approx(sol[1], rel=1e-10, abs=1e-12)
        assert chi2[k] == pytest.approx(res[0], rel=1e-10)
    F = 1.7 * a[0] + 0.3
    chi2, Fs, Fb, deg = fit_and_chi2(a[:1], F, w)
    assert Fs[0] == pytest.approx(1.7, rel=1e-12) and Fb[0] == pytest.approx(0.3, rel=1e-10)
    assert chi2[0] < 1e-18 * np.sum(w * F * F)


def test_degenerate_fit():
    a = np.full((1, 50), 2.5)
    F = np.linspace(1, 2, 50)
    w = np.ones(50)
    chi2, Fs, Fb, deg = fit_and_chi2(a, F, w)
    assert deg[0] and Fs[0] == 0.0 and Fb[0] == pytest.approx(F.mean(), rel=1e-14)
    assert chi2[0] == pytest.approx(np.sum((F - F.mean()) ** 2), rel=1e-12)


def test_neumaier_matches_fsum():
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (3, 5000)) * 10 ** rng.uniform(-8, 8, (3, 5000))
    s = neumaier_sum(x)
    for k in range(3):
        assert s[k] == pytest.approx(math.fsum(x[k]), rel=1e-15, abs=1e-300)


def test_topk_order_ties_and_nan():
    c = np.array([3.0, np.nan, 1.0, 3.0, 0.5, np.nan, 1.0])
    idx, val = topk(c, 7)
    assert list(idx) == [4, 2, 6, 0, 3, 1, 5]
    idx, val = topk(c, 3)
    assert list(idx) == [4, 2, 6]


def _pure_python_chi2(amap, window, t, F, w, p):
    """Brute force in pure-Python FP64 (math.fsum), bilinear on pixel centres."""
    cx, cy, vx, vy, mx, my = window
    t0, u0, tE, al = p
    ca, sa = math.cos(al), math.sin(al)
    A = []
    for ti in t:
        tau = (ti - t0) / tE
        zx, zy = tau * ca - u0 * sa, tau * sa + u0 * ca
        gx = (zx - cx) * mx / vx + mx / 2 - 0.5
        gy = (zy - cy) * my / vy + my / 2 - 0.5
        if 0 <= gx < mx - 1 and 0 <= gy < my - 1:
            i, j = int(math.floor(gx)), int(math.floor(gy))
            fx, fy = gx - i, gy - j
            v = [[float(amap[j + bb, i + aa]) for aa in (0, 1)] for bb in (0, 1)]
            A.append((1 - fx) * (1 - fy) * v[0][0] + fx * (1 - fy) * v[0][1]
                     + (1 - fx) * fy * v[1][0] + fx * fy * v[1][1])
        else:
            u = math.hypot(zx, zy)
            A.append((u * u + 2) / (u * math.sqrt(u * u + 4)))
    Sw = math.fsum(w)
    SA = math.fsum(wi * ai for wi, ai in zip(w, A))
    SAA = math.fsum(wi * ai * ai for wi, ai in zip(w, A))
    SF = math.fsum(wi * fi for wi, fi in zip(w, F))
    SAF = math.fsum(wi * ai * fi for wi, ai, fi in zip(w, A, F))
    det = SAA * Sw - SA * SA
    Fs = (SAF * Sw - SA * SF) / det
    Fb = (SAA * SF - SA * SAF) / det
    return math.fsum(wi * (fi - Fs * ai - Fb) ** 2 for wi, ai, fi in zip(w, A, F))


def test_brute_force_tiny_grid_and_truth_chi2():
    """Paczynski map + single-lens data: exact64 search equals pure-Python brute force,
    and chi2 at the truth is consistent with N +- a few sqrt(2N)."""
    win = (0.0, 0.0, 2.0, 2.0, 256, 256)
    d = 2.0 / 256
    c = -1 + (np.arange(256) + 0.5) * d
    amap = paczynski(np.hypot(c[None, :], c[:, None])).astype(np.float32)
    rng = np.random.default_rng(8)
    n = 200
    t = np.sort(rng.uniform(-40, 40, n))
    truth = np.array([0.0, 0.3, 20.0, 0.6])
    z = trajectory_positions(truth, t)
    Ftrue = 1.0 * paczynski(np.abs(z)) + 0.2
    sig = 0.01 * Ftrue
    F = Ftrue + sig * rng.standard_normal(n)
    w = 1 / sig ** 2
    params = grid_params([0.25, 0.3, 0.35], [0.5, 0.6, 0.7], [-1.0, 0.0], [20.0, 22.0])
    chi2, Fs, Fb, _ = search_exact64(amap, win, t, F, w, params)
    for k in range(len(params)):
        assert chi2[k] == pytest.approx(_pure_python_chi2(amap, win, t, F, w, params[k]), rel=1e-9)
    best = np.argmin(chi2)
    # a single-lens map is rotationally symmetric: alpha is degenerate
    assert np.allclose(params[best][:3], truth[:3])
    at_truth = np.flatnonzero(np.all(np.isclose(params, truth), axis=1))[0]
    assert abs(chi2[at_truth] - n) < 5 * math.sqrt(2 * n)
    c32, _, _, _ = search_mirror32(amap, win, (t - 0.0).astype(np.float32), F, w, params, 0.0)
    assert np.abs(c32 / chi2 - 1).max() < 1e-3
