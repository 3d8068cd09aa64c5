"""Profiled linear flux fit, chi-square and selection (test infrastructure only).

Eq. 5: F_i = F_S A(t_i) + F_B; Eq. 6: the (difference) flux is linear in A, so for a
given trajectory the two flux parameters have a closed-form weighted least-squares
solution, the unconstrained minimiser (no sign constraint).  With weights w_i = 1/sigma_i^2
and a_i = A(t_i) promoted to FP64 it is computed from the centred normal equations:
    S_w = sum w,  abar = sum w a / S_w,  Fbar = sum w F / S_w,
    S_aa = sum w (a - abar)^2,  S_aF = sum w (a - abar)(F - Fbar),
    F_s = S_aF / S_aa,  F_b = Fbar - F_s abar,
the same minimiser as (S_AF S_w - S_A S_F)/det, (S_AA S_F - S_A S_AF)/det with
det = S_AA S_w - S_A^2 = S_w S_aa, written without the cancellation of det when a is
nearly constant.  When det <= 1e-12 S_AA S_w (i.e. S_aa <= 1e-12 S_AA, S_AA = sum w a^2)
the magnification is numerically constant and the fit degenerates:
F_s = 0, F_b = Fbar.  Chi-square (sec. 4.2: sum of per-point contributions) is summed
directly, chi2 = sum w (F - F_s a - F_b)^2, over the same a.

All sums here use Neumaier-compensated FP64 summation over the points, vectorised
across trajectories.  Selection (sec. 4.4, best solutions as seeds) orders by
(chi2, index), NaN last.
"""
from __future__ import annotations

import numpy as np

__all__ = ["neumaier_sum", "normal_sums", "profiled_fit", "chi2_direct", "fit_and_chi2",
           "topk", "DEGENERATE_RTOL"]

DEGENERATE_RTOL = 1e-12


def neumaier_sum(x, axis=-1):
    """Compensated sum of FP64 values along ``axis`` (Neumaier's variant of Kahan)."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    s = np.zeros(x.shape[:-1])
    c = np.zeros(x.shape[:-1])
    for k in range(x.shape[-1]):
        v = x[..., k]
        t = s + v
        big = np.abs(s) >= np.abs(v)
        c += np.where(big, (s - t) + v, (v - t) + s)
        s = t
    return s + c


def normal_sums(a, F, w):
    """Weighted sums of the fit (last axis = points): S_w, S_A, S_AA, S_F, S_AF and the
    centred abar, Fbar, S_aa, S_aF."""
    a = np.asarray(a, dtype=np.float64)
    F = np.broadcast_to(np.asarray(F, dtype=np.float64), a.shape)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), a.shape)
    Sw = neumaier_sum(w)
    SA = neumaier_sum(w * a)
    SF = neumaier_sum(w * F)
    abar = SA / Sw
    Fbar = SF / Sw
    da = a - abar[..., None]
    dF = F - Fbar[..., None]
    return dict(Sw=Sw, SA=SA, SAA=neumaier_sum(w * a * a), SF=SF, SAF=neumaier_sum(w * a * F),
                abar=abar, Fbar=Fbar, Saa=neumaier_sum(w * da * da), SaF=neumaier_sum(w * da * dF))


def profiled_fit(sums):
    """(Fs, Fb, degenerate) from ``normal_sums`` (centred form, see the module doc)."""
    Sw, SAA, Saa, SaF, abar, Fbar = (sums[k] for k in ("Sw", "SAA", "Saa", "SaF", "abar", "Fbar"))
    degenerate = ~(Saa > DEGENERATE_RTOL * SAA)
    with np.errstate(divide="ignore", invalid="ignore"):
        Fs = np.where(degenerate, 0.0, SaF / Saa)
        Fb = np.where(degenerate, Fbar, Fbar - Fs * abar)
    return Fs, Fb, degenerate


def chi2_direct(a, F, w, Fs, Fb):
    a = np.asarray(a, dtype=np.float64)
    r = np.asarray(F)[None, :] - np.asarray(Fs)[:, None] * a - np.asarray(Fb)[:, None]
    return neumaier_sum(np.asarray(w)[None, :] * r * r)


def fit_and_chi2(a, F, w):
    """a [n_traj, n_pts] -> (chi2, Fs, Fb, degenerate) per trajectory."""
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    sums = normal_sums(a, F[None, :], w[None, :])
    Fs, Fb, deg = profiled_fit(sums)
    return chi2_direct(a, F, w, Fs, Fb), Fs, Fb, deg


def topk(chi2, k):
    """Indices and values of the k smallest chi2, ordered by (chi2, index), NaN last."""
    c = np.asarray(chi2, dtype=np.float64).reshape(-1)
    idx = np.arange(c.size)
    isn = np.isnan(c)
    order = np.lexsort((idx, np.where(isn, 0.0, c), isn))
    sel = order[:k]
    return sel.astype(np.int64), c[sel]
