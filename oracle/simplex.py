"""Downhill-simplex search along caustic-centred lines (test infrastructure only).

Sec. 4.2: for each (r, phi) trajectory (a line, see ``lines``) and map, the paper runs
a downhill simplex (Nelder & Mead 1965) for the chi-square minimum, with up to 5000 steps
(sec. 5).  Readings fixed here:
  * the simplex runs over x = (t0', ln tE) (t0' = time of closest approach to the
    caustic centre; ln tE keeps tE positive), one simplex per (line, map): the source
    radius is the map index of a finite-source stack rather than a continuous simplex
    coordinate;
  * start x0 and the initial vertices x0 + (d_t0, 0), x0 + (0, d_ln_tE);
  * the standard coefficients (reflection 1, expansion 2, contraction 1/2, shrink 1/2)
    with the acceptance rules of Lagarias et al. (1998): reflect; if better than the
    best, expand and keep the better of the two; if between the best and the
    second-worst, keep the reflection; else contract outside (reflection better than
    the worst: keep if not worse than the reflection) or inside (keep if better than the
    worst), and otherwise shrink towards the best vertex;
  * vertices ordered by chi-square with a stable sort, a new vertex ranking after old
    ones of equal value; NaN counts as +inf;
  * stop when f_worst - f_best <= ftol |f_best| or after max_iter iterations;
  * FP64 vertex arithmetic in the order written below; chi-square of a vertex is the
    search's chi-square (binary32 samples, profiled FP64 fit) of the trajectory
    (t0' - shift tE, u0, tE, alpha), its sums taken exactly rounded (math.fsum), as
    one trajectory at a time is evaluated.
"""
from __future__ import annotations

import math

import numpy as np

from .sampling import sample_mirror32, traj_constants32

__all__ = ["nelder_mead", "line_chi2", "line_simplex"]


def _key(f):
    return math.inf if f != f else f


def nelder_mead(func, x0, steps, max_iter=5000, ftol=1e-10):
    """Minimise func over R^2 from x0; returns (x_best, f_best, iterations, evaluations)."""
    calls = [0]

    def fn(v):
        calls[0] += 1
        return _key(func(v))

    x = [list(map(float, x0)), [float(x0[0]) + float(steps[0]), float(x0[1])],
         [float(x0[0]), float(x0[1]) + float(steps[1])]]
    f = [fn(v) for v in x]

    def order():
        idx = sorted(range(3), key=lambda i: f[i])  # stable: equal values keep their order
        x[:] = [x[i] for i in idx]
        f[:] = [f[i] for i in idx]

    def replace(v, fv):
        x[2] = v
        f[2] = fv
        order()

    order()
    it = 0
    while it < max_iter and not (f[2] - f[0] <= ftol * abs(f[0])):
        it += 1
        xb = [(x[0][k] + x[1][k]) * 0.5 for k in range(2)]
        xr = [xb[k] + (xb[k] - x[2][k]) for k in range(2)]
        fr = fn(xr)
        if fr < f[0]:
            xe = [xb[k] + 2.0 * (xb[k] - x[2][k]) for k in range(2)]
            fe = fn(xe)
            if fe < fr:
                replace(xe, fe)
            else:
                replace(xr, fr)
        elif fr < f[1]:
            replace(xr, fr)
        else:
            if fr < f[2]:
                xc = [xb[k] + 0.5 * (xr[k] - xb[k]) for k in range(2)]
                fc = fn(xc)
                ok = fc <= fr
            else:
                xc = [xb[k] + 0.5 * (x[2][k] - xb[k]) for k in range(2)]
                fc = fn(xc)
                ok = fc < f[2]
            if ok:
                replace(xc, fc)
            else:
                for i in (1, 2):
                    x[i] = [x[0][k] + 0.5 * (x[i][k] - x[0][k]) for k in range(2)]
                    f[i] = fn(x[i])
                order()
    return x[0], f[0], it, calls[0]


def _chi2_one(A, F, w):
    """Profiled chi-square of one trajectory (Eqs. 5-6 in the centred form of the search,
    degenerate when S_aa <= 1e-12 S_AA), every sum exactly rounded (math.fsum)."""
    a = np.asarray(A, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    Sw = math.fsum(w)
    abar = math.fsum(w * a) / Sw
    Fbar = math.fsum(w * F) / Sw
    SAA = math.fsum(w * a * a)
    da = a - abar
    Saa = math.fsum(w * da * da)
    if Saa > 1e-12 * SAA:
        Fs = math.fsum(w * da * (F - Fbar)) / Saa
        Fb = Fbar - Fs * abar
    else:
        Fs, Fb = 0.0, Fbar
    r = F - Fs * a - Fb
    return math.fsum(w * r * r)


def line_chi2(amap, window, tt, F, w, t_ref, line, x):
    """Chi-square of the line's trajectory at x = (t0', ln tE)."""
    u0, al, shift = (float(v) for v in line)
    tE = math.exp(x[1])
    p = np.array([[x[0] - shift * tE, u0, tE, al]])
    A = sample_mirror32(amap, window, traj_constants32(p, t_ref), tt)[0]
    return _chi2_one(A, F, w)


def line_simplex(amap, window, tt, F, w, t_ref, line, start, steps, max_iter=5000, ftol=1e-10):
    """Simplex endpoint of one line: (t0', tE, chi2, iterations, evaluations) from start
    (t0', tE)."""
    x, f, it, ne = nelder_mead(lambda v: line_chi2(amap, window, tt, F, w, t_ref, line, v),
                           (float(start[0]), math.log(float(start[1]))), steps, max_iter, ftol)
    return x[0], math.exp(x[1]), f, it, ne
