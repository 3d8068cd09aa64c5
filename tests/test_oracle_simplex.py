"""Pins of oracle.simplex: the downhill simplex (Nelder & Mead 1965, Lagarias et al.
1998 acceptance rules) and its use along a line (sec. 4.2)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle.lens import paczynski
from oracle.simplex import line_chi2, line_simplex, nelder_mead


def test_quadratic_minimum():
    f = lambda v: (v[0] - 1.0) ** 2 + 10.0 * (v[1] + 2.0) ** 2
    x, fx, it, ne = nelder_mead(f, (4.0, 3.0), (0.5, 0.5), max_iter=2000, ftol=1e-14)
    assert 3 + it <= ne <= 3 + 4 * it
    assert abs(x[0] - 1.0) < 1e-5 and abs(x[1] + 2.0) < 1e-5 and fx < 1e-10 and it < 2000


def test_rosenbrock_agrees_with_scipy():
    f = lambda v: 100.0 * (v[1] - v[0] ** 2) ** 2 + (1.0 - v[0]) ** 2
    x, fx, it, _ = nelder_mead(f, (-1.2, 1.0), (0.1, 0.1), max_iter=5000, ftol=1e-15)
    ref = optimize.minimize(f, (-1.2, 1.0), method="Nelder-Mead",
                            options=dict(xatol=1e-10, fatol=1e-15, maxiter=5000))
    assert abs(x[0] - 1.0) < 1e-4 and abs(x[1] - 1.0) < 1e-4
    assert np.allclose(x, ref.x, atol=1e-4)


def test_iteration_cap_and_nan_as_infinity():
    calls = []

    def f(v):
        calls.append(1)
        return float("nan") if v[0] > 2.0 else (v[0] - 1.0) ** 2 + v[1] ** 2

    x, fx, it, ne = nelder_mead(f, (0.0, 0.5), (1.5, 0.3), max_iter=7, ftol=0.0)
    assert it == 7 and math.isfinite(fx) and fx <= (0.0 - 1.0) ** 2 + 0.25
    assert ne == len(calls)


def test_line_simplex_recovers_single_lens_truth():
    # q = 0 map filled with the single-lens magnification; noise-free data of a
    # trajectory with u0 = 0.2 along alpha = 0.7: the simplex over (t0', ln tE) from a
    # displaced start finds t0 = 3, tE = 25
    nx = 1024
    win = (0.0, 0.0, 4.0, 4.0, nx, nx)
    d = 4.0 / nx
    xs = (np.arange(nx) - nx / 2 + 0.5) * d
    amap = paczynski(np.hypot(xs[None, :], xs[:, None])).astype(np.float32)
    u0, al, t0, tE = 0.2, 0.7, 3.0, 25.0
    t = np.sort(np.random.default_rng(4).uniform(-45, 45, 400))
    tau = (t - t0) / tE
    A = paczynski(np.hypot(tau, u0))
    F = 1.0 * A + 0.2
    w = np.full_like(t, 1e4)
    tt = t.astype(np.float32)
    line = (u0, al, 0.0)
    assert line_chi2(amap, win, tt, F, w, 0.0, line, (t0, math.log(tE))) < 1e-2
    t0f, tEf, chi2, it, _ = line_simplex(amap, win, tt, F, w, 0.0, line, (0.0, 15.0), (2.0, 0.2),
                                      max_iter=2000, ftol=1e-12)
    assert abs(t0f - t0) < 2e-3 and abs(tEf / tE - 1) < 1e-3 and chi2 < 1e-2


def test_line_chi2_equals_the_search_chi2():
    from oracle.search import search_mirror32
    rng = np.random.default_rng(8)
    nx = 256
    win = (0.0, 0.0, 2.0, 2.0, nx, nx)
    amap = (1.0 + rng.random((nx, nx))).astype(np.float32)
    t = np.sort(rng.uniform(-30, 30, 300))
    F = 1.0 + rng.random(300)
    w = 1.0 / (0.01 + 0.01 * rng.random(300)) ** 2
    tt = (t - 5.0).astype(np.float32)
    for line, x in (((0.1, 0.4, 0.2), (1.0, math.log(18.0))), ((0.6, 2.5, -0.3), (-4.0, math.log(40.0)))):
        u0, al, shift = line
        tE = math.exp(x[1])
        ref = search_mirror32(amap, win, tt, F, w, np.array([[x[0] - shift * tE, u0, tE, al]]), 5.0)[0][0]
        assert line_chi2(amap, win, tt, F, w, 5.0, line, x) == pytest.approx(ref, rel=1e-12)
