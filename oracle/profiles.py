"""Limb-darkened source-profile weights for finite-source maps (test infrastructure only).

Sec. 4.1 of the paper convolves each point-source magnification map with radially
symmetric source intensity profiles of several radii rho and one fixed limb-darkening
coefficient (Gamma_I = 0.53), giving a stack of finite-source maps, one per rho (seven
rho log-spaced over (0.001, 1)).  The profile read here is the linear limb-darkening law
in its Gamma form, normalised to unit mean surface brightness over the disk:

    I(r) = 1 - Gamma (1 - (3/2) sqrt(1 - r^2/rho^2)),   0 <= r <= rho,

whose integral over the disk is pi rho^2 for every Gamma (the mean of
sqrt(1 - r^2/rho^2) over the disk is 2/3).  Gamma = 0 is the uniform disk.

The finite-source value at a pixel centre is the profile-weighted average of the
piecewise-constant count density, so the weight of the pixel at offset (a, b) is

    w[b, a] = (integral of I over pixel(a, b) ∩ disk) / (pi rho^2).

This oracle evaluates that integral by quadrature: for fixed x the integral over y has
the closed form (1 - Gamma)(yb - ya) + (3 Gamma/(2 rho)) [S(yb) - S(ya)] with
S(y) = (y sqrt(c^2 - y^2) + c^2 asin(y/c))/2 and c = sqrt(rho^2 - x^2); the x integral
is split where the chord half-length c crosses the pixel's y edges or vanishes, and
each piece is integrated with Gauss-Legendre nodes after the substitution
x = p + (q - p)(1 - cos theta)/2, which removes the square-root behaviour at the piece
ends.  The weights are then renormalised to sum 1, like the uniform-disk weights.
"""
from __future__ import annotations

import math

import numpy as np

from .maps import stencil_radius

__all__ = ["ld_intensity", "ld_pixel_weights", "ld_rect_integral", "stack_rhos"]

_NODES, _WEIGHTS = np.polynomial.legendre.leggauss(48)


def ld_intensity(r, rho: float, gamma: float):
    """Surface brightness I(r) of the linear law (unit mean over the disk); 0 outside."""
    r = np.asarray(r, dtype=np.float64)
    inside = r <= rho
    mu = np.sqrt(np.clip(1.0 - (r / rho) ** 2, 0.0, None))
    return np.where(inside, 1.0 - gamma * (1.0 - 1.5 * mu), 0.0)


def _inner(x, y1, y2, rho, gamma):
    """Integral over y in [y1, y2] of I(sqrt(x^2 + y^2)) for an array of x."""
    c2 = np.clip(rho * rho - x * x, 0.0, None)
    c = np.sqrt(c2)
    ya = np.maximum(y1, -c)
    yb = np.minimum(y2, c)
    ok = yb > ya

    def S(y):  # antiderivative of sqrt(c^2 - y^2); (c - y)(c + y) is exactly 0 at y = +-c
        cs = np.where(c > 0, c, 1.0)
        return 0.5 * (y * np.sqrt(np.clip((c - y) * (c + y), 0.0, None))
                      + c2 * np.arcsin(np.clip(y / cs, -1.0, 1.0)))

    val = (1.0 - gamma) * (yb - ya) + (1.5 * gamma / rho) * (S(yb) - S(ya))
    return np.where(ok, val, 0.0)


def ld_rect_integral(x1, x2, y1, y2, rho: float, gamma: float):
    """Integral of I over [x1, x2] x [y1, y2] ∩ disk(0, rho), elementwise over arrays of
    rectangles (scalars give a scalar)."""
    x1, x2, y1, y2 = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x1, x2, y1, y2)))
    shape = x1.shape
    x1, x2, y1, y2 = (v.reshape(-1) for v in (x1, x2, y1, y2))
    lo = np.maximum(x1, -rho)
    hi = np.minimum(x2, rho)
    # cut points: the piece ends plus +-sqrt(rho^2 - y^2) for each y edge inside the disk
    cand = [lo, hi]
    for y in (y1, y2):
        xc = np.sqrt(np.clip(rho * rho - y * y, 0.0, None))
        inside = np.abs(y) < rho
        for xv in (-xc, xc):
            cand.append(np.where(inside, np.clip(xv, lo, hi), lo))
    cuts = np.sort(np.stack(cand, axis=1), axis=1)  # [n, 6]
    th = 0.5 * math.pi * (_NODES + 1.0)  # theta in (0, pi)
    total = np.zeros(x1.shape)
    for k in range(cuts.shape[1] - 1):
        p, q = cuts[:, k:k + 1], cuts[:, k + 1:k + 2]
        x = p + 0.5 * (q - p) * (1.0 - np.cos(th))[None, :]
        jac = 0.5 * (q - p) * (np.sin(th) * 0.5 * math.pi)[None, :]
        val = _inner(x, y1[:, None], y2[:, None], rho, gamma)
        total += np.sum(_WEIGHTS[None, :] * jac * val, axis=1)
    total = np.where(hi > lo, total, 0.0)
    return total.reshape(shape) if shape else float(total[0])


def ld_pixel_weights(rho: float, dx: float, dy: float, gamma: float, normalise: bool = True):
    """FP64 weights [2Ry+1, 2Rx+1] (row = y offset) of the limb-darkened disk.

    rho = 0 gives the identity; the stencil radius is the uniform disk's,
    R = ceil(rho/d + 1/2), with all-zero outer rings trimmed.  normalise=False returns
    the raw integrals over pi rho^2 (their sum is 1 up to quadrature error)."""
    if rho <= 0.0:
        return np.ones((1, 1))
    Rx = stencil_radius(rho, dx)
    Ry = stencil_radius(rho, dy)
    # the weights are even in a and in b: integrate the quadrant a, b >= 0 and mirror
    a = np.arange(Rx + 1, dtype=np.float64)[None, :]
    b = np.arange(Ry + 1, dtype=np.float64)[:, None]
    quad = np.zeros((Ry + 1, Rx + 1))
    for j0 in range(0, Ry + 1, 64):  # rows in chunks (bounded memory)
        bb = b[j0:j0 + 64]
        quad[j0:j0 + 64] = ld_rect_integral((a - 0.5) * dx, (a + 0.5) * dx, (bb - 0.5) * dy,
                                            (bb + 0.5) * dy, rho, gamma)
    # a pixel that does not meet the open disk has weight 0 exactly (as for the uniform disk)
    nxd = np.maximum(0.0, (a - 0.5) * dx)
    nyd = np.maximum(0.0, (b - 0.5) * dy)
    quad[nxd * nxd + nyd * nyd >= rho * rho] = 0.0
    w = np.concatenate([quad[:0:-1], quad], axis=0)
    w = np.concatenate([w[:, :0:-1], w], axis=1)
    w /= math.pi * rho * rho
    if normalise:
        w /= w.sum()
    while w.shape[0] > 1 and not w[0].any() and not w[-1].any():
        w = w[1:-1]
    while w.shape[1] > 1 and not w[:, 0].any() and not w[:, -1].any():
        w = w[:, 1:-1]
    return w


def stack_rhos(n: int = 7, lo: float = 1e-3, hi: float = 1.0):
    """The stack's source radii: n values log-spaced over [lo, hi], endpoints included."""
    return np.logspace(math.log10(lo), math.log10(hi), n)
