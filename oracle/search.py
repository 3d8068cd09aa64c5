"""Brute-force trajectory search over a map (test infrastructure only).

Sec. 4.2: each trajectory through a (d, q, rho) map is scored against the light
curve; sec. 4.4: the best solutions seed the next stage.  The oracle evaluates the
plain definition for every trajectory: sample the map along the trajectory
(``sampling``), profile (F_s, F_b) and sum chi-square (``fit``).

Trajectory order for a product grid: row-major over
(u0, alpha, t0, tE), i.e. index = ((iu0 * n_alpha + ia) * n_t0 + it0) * n_tE + itE.
Parameters are rows (t0, u0, tE, alpha) in FP64.
"""
from __future__ import annotations

import numpy as np

from .sampling import traj_constants32, sample_mirror32, sample_exact64
from .fit import fit_and_chi2

__all__ = ["grid_params", "search_mirror32", "search_exact64"]


def grid_params(u0s, alphas, t0s, tEs):
    U, AL, T0, TE = np.meshgrid(np.asarray(u0s, float), np.asarray(alphas, float),
                                np.asarray(t0s, float), np.asarray(tEs, float), indexing="ij")
    return np.stack([T0.ravel(), U.ravel(), TE.ravel(), AL.ravel()], axis=1)


def search_mirror32(amap, window, tt, F, w, params, t_ref, chunk=256):
    """chi2, Fs, Fb, degenerate for each row of params (binary32 sampling, FP64 fit)."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    out = [np.empty(len(params)) for _ in range(3)] + [np.empty(len(params), bool)]
    for a in range(0, len(params), chunk):
        b = min(a + chunk, len(params))
        A = sample_mirror32(amap, window, traj_constants32(params[a:b], t_ref), tt)
        res = fit_and_chi2(A.astype(np.float64), F, w)
        for o, r in zip(out, res):
            o[a:b] = r
    return tuple(out)


def search_exact64(amap, window, t, F, w, params, t_ref=0.0, chunk=256):
    params = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    out = [np.empty(len(params)) for _ in range(3)] + [np.empty(len(params), bool)]
    for a in range(0, len(params), chunk):
        b = min(a + chunk, len(params))
        A = sample_exact64(amap, window, params[a:b], t, t_ref)
        res = fit_and_chi2(A, F, w)
        for o, r in zip(out, res):
            o[a:b] = r
    return tuple(out)
