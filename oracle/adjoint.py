"""Chi-square gradient with respect to (t0, u0, tE, alpha) (test infrastructure only).

The objective is the profiled chi-square of ``fit`` evaluated on map samples along
the trajectory (sec. 4.2).  Because (F_s, F_b) are the exact minimisers for the given
samples, the envelope theorem gives
    d chi2 / d theta = -2 F_s sum_i w_i r_i d a_i / d theta,   r = F - F_s a - F_b,
(the F_s, F_b derivatives drop out since sum w r a = sum w r = 0).  ``chi2_grad_explicit``
differentiates through the 2x2 solve instead; the two must agree (pin).

d a / d theta follows the sampling chain of ``sampling``:
  on map: dA/dgx = e0 + fy (e1 - e0), dA/dgy = ax1 - ax0, dA/dzeta = k dA/dg;
  off map: A(u) = (u^2+2)/(u sqrt(u^2+4)), dA/du = -8/(u^2 (u^2+4)^(3/2)), du/dzeta = zeta/u;
  zeta = tau (ca, sa) + u0 (-sa, ca), tau = (t - t0)/tE:
  d zeta/d t0 = -(ca, sa)/tE, d zeta/d tE = -tau (ca, sa)/tE, d zeta/d u0 = (-sa, ca),
  d zeta/d alpha = (-zeta_y, zeta_x).
In the mirror32 mode every per-point quantity is the binary32 sample quantity promoted
to FP64, and all products and sums are FP64.
"""
from __future__ import annotations

import numpy as np

from .sampling import traj_constants32, sample_mirror32, sample_exact64
from .fit import normal_sums, profiled_fit, chi2_direct, neumaier_sum, fit_and_chi2

__all__ = ["sample_derivatives", "chi2_grad", "chi2_grad_explicit", "chi2_exact64",
           "fd_gradient"]


def sample_derivatives(amap, window, params, tt=None, t=None, t_ref=0.0, mode="mirror32"):
    """Returns (a [n, m] FP64, da [4, n, m] FP64) for theta = (t0, u0, tE, alpha)."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    if mode == "mirror32":
        k = traj_constants32(params, t_ref)
        A, P = sample_mirror32(amap, window, k, tt, parts=True)
        ca = k["ca"].astype(np.float64)[:, None]
        sa = k["sa"].astype(np.float64)[:, None]
    else:
        A, P = sample_exact64(amap, window, params, t, t_ref, parts=True)
        ca = np.cos(params[:, 3])[:, None]
        sa = np.sin(params[:, 3])[:, None]
    d = {n: np.asarray(v, dtype=np.float64) if isinstance(v, np.ndarray) else float(v)
         for n, v in P.items() if n not in ("onmap", "i0", "j0")}
    on = P["onmap"]
    dgx = d["e0"] + d["fy"] * (d["e1"] - d["e0"])
    dgy = d["ax1"] - d["ax0"]
    zx, zy = d["zx"], d["zy"]
    with np.errstate(divide="ignore", invalid="ignore"):
        u2 = zx * zx + zy * zy
        u = np.sqrt(u2)
        dAdu = -8.0 / (u2 * (u2 + 4.0) ** 1.5)
        offx = dAdu * zx / u
        offy = dAdu * zy / u
    dAx = np.where(on, d["kx"] * dgx, offx)
    dAy = np.where(on, d["ky"] * dgy, offy)
    tE = params[:, 2][:, None]
    tau = d["tau"]
    da = np.stack([
        dAx * (-ca / tE) + dAy * (-sa / tE),
        dAx * (-sa) + dAy * ca,
        dAx * (-tau * ca / tE) + dAy * (-tau * sa / tE),
        dAx * (-zy) + dAy * zx,
    ])
    return A.astype(np.float64), da


def chi2_grad(amap, window, tt, F, w, params, t_ref=0.0, t=None, mode="mirror32"):
    """Envelope-form gradient.  Returns (chi2 [n], grad [n, 4], Fs [n], Fb [n])."""
    a, da = sample_derivatives(amap, window, params, tt=tt, t=t, t_ref=t_ref, mode=mode)
    sums = normal_sums(a, F[None, :], w[None, :])
    Fs, Fb, _ = profiled_fit(sums)
    r = F[None, :] - Fs[:, None] * a - Fb[:, None]
    chi2 = neumaier_sum(w[None, :] * r * r)
    wr = w[None, :] * r
    grad = np.stack([-2.0 * Fs * neumaier_sum(wr * da[k]) for k in range(4)], axis=1)
    return chi2, grad, Fs, Fb


def chi2_grad_explicit(amap, window, tt, F, w, params, t_ref=0.0):
    """Gradient by differentiating the 2x2 solve explicitly (mirror32 samples)."""
    a, da = sample_derivatives(amap, window, params, tt=tt, t_ref=t_ref)
    W = w[None, :]
    Sw, SA, SAA = neumaier_sum(W * np.ones_like(a)), neumaier_sum(W * a), neumaier_sum(W * a * a)
    SF, SAF = neumaier_sum(W * F[None, :] * np.ones_like(a)), neumaier_sum(W * a * F[None, :])
    det = SAA * Sw - SA * SA
    Fs = (SAF * Sw - SA * SF) / det
    Fb = (SAA * SF - SA * SAF) / det
    r = F[None, :] - Fs[:, None] * a - Fb[:, None]
    grads = []
    for k in range(4):
        dSA = neumaier_sum(W * da[k])
        dSAA = neumaier_sum(2.0 * W * a * da[k])
        dSAF = neumaier_sum(W * da[k] * F[None, :])
        ddet = dSAA * Sw - 2.0 * SA * dSA
        nFs = SAF * Sw - SA * SF
        nFb = SAA * SF - SA * SAF
        dFs = ((dSAF * Sw - dSA * SF) * det - nFs * ddet) / (det * det)
        dFb = ((dSAA * SF - dSA * SAF) * det - nFb * ddet) / (det * det)
        dr = -dFs[:, None] * a - Fs[:, None] * da[k] - dFb[:, None]
        grads.append(neumaier_sum(2.0 * W * r * dr))
    return np.stack(grads, axis=1)


def chi2_exact64(amap, window, t, F, w, params, t_ref=0.0):
    A = sample_exact64(amap, window, params, t, t_ref)
    return fit_and_chi2(A, F, w)[0]


def fd_gradient(amap, window, t, F, w, params, t_ref=0.0, rel=1e-5, mode="exact64", tt=None):
    """Central differences of the chi-square objective.

    mode "exact64": FP64 sampling from absolute times t; mode "mirror32": the
    binary32 sampling of the search (times tt = fl32(t - t_ref)), i.e. the objective
    the refinement minimises.  Step h = rel * max(|theta|, s_theta),
    s = (tE, 1e-2, tE, 1), except for t0: a position in time, whose step is rel * tE
    whatever the calendar origin (with absolute dates |t0| ~ 2.5e6 d, a step relative
    to |t0| would span weeks of the light curve).  A component is eligible only when no sample changes
    bilinear cell or on/off-map state between theta - h and theta + h (the bilinear
    interpolant has kinks at cell edges).  Returns (fd [n, 4], eligible [n, 4]).
    """
    params = np.asarray(params, dtype=np.float64).reshape(-1, 4)

    def evaluate(p):
        if mode == "exact64":
            return sample_exact64(amap, window, p, t, t_ref, parts=True)
        return sample_mirror32(amap, window, traj_constants32(p, t_ref), tt, parts=True)

    n = len(params)
    fd = np.zeros((n, 4))
    elig = np.zeros((n, 4), dtype=bool)
    for k in range(4):
        scale = np.stack([params[:, 2], np.full(n, 1e-2), params[:, 2], np.ones(n)], axis=1)[:, k]
        h = rel * (params[:, 2] if k == 0 else np.maximum(np.abs(params[:, k]), scale))
        pp = params.copy()
        pm = params.copy()
        pp[:, k] += h
        pm[:, k] -= h
        Ap, Pp = evaluate(pp)
        Am, Pm = evaluate(pm)
        cp = fit_and_chi2(np.asarray(Ap, np.float64), F, w)[0]
        cm = fit_and_chi2(np.asarray(Am, np.float64), F, w)[0]
        fd[:, k] = (cp - cm) / (2.0 * h)
        same = (Pp["onmap"] == Pm["onmap"]) & (Pp["i0"] == Pm["i0"]) & (Pp["j0"] == Pm["j0"])
        elig[:, k] = same.all(axis=1)
    return fd, elig
