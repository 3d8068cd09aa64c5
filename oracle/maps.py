"""Count normalisation and uniform-disk convolution (test infrastructure only).

Sec. 4.1 of the paper convolves each point-source map with radially symmetric source
profiles of radius rho to obtain finite-source maps.  Here the profile is the uniform
disk (no limb darkening) and the map is the piecewise-constant ray-count density of
``rays``; the finite-source value at a pixel centre is the average of the
count density over the disk of radius rho about that centre, i.e. a weighted sum of
the neighbouring pixels with weights w = area(disk ∩ pixel) / (pi rho^2).

Normalisation: with lattice spacing (hx, hy) the unlensed ray density is 1/(hx hy)
rays per unit area, so a pixel of area dx*dy holds dx*dy/(hx*hy) rays at magnification
1 and A = count * (hx*hy)/(dx*dy).

FP32 mirror: scale = fl32(hx32*hy32/(dx*dy)) computed in FP64 from
the binary32 lattice spacings; weights computed in FP64, renormalised to sum 1,
rounded once; taps visited row-major (dy outer, dx inner) over the (2Ry+1)x(2Rx+1)
stencil, R = ceil(rho/d + 1/2), zero taps skipped; acc = ((w0*c0) + (w1*c1)) + ...
in binary32; neighbours beyond the window edge take the edge pixel (clamp);
A = acc * scale.  The exact64 variant does the same in FP64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["disk_pixel_weights", "map_scale", "normalize_convolve_mirror32",
           "normalize_convolve_exact64", "normalize_convolve_exact64_at", "stencil_radius"]


def _seg_area(x, y, R):
    """Area of {(X, Y): X^2 + Y^2 <= R^2, X <= x, Y <= y} for a disk of radius R.

    Written as the integral over X of the length of {Y <= y} within the chord at X.
    For |y| < R the chord at X is cut by Y = y only for |X| <= w = sqrt(R^2 - y^2):
      y >= 0: length 2h(X) for |X| > w, y + h(X) for |X| <= w;
      y < 0 : length y + h(X) for |X| <= w, 0 otherwise;
    with h(X) = sqrt(R^2 - X^2) and H(X) = (X h(X) + R^2 asin(X/R))/2 its antiderivative.
    """
    if y <= -R or x <= -R:
        return 0.0
    xe = min(x, R)

    def H(t):
        t = max(-R, min(R, t))
        return 0.5 * (t * math.sqrt(max(R * R - t * t, 0.0)) + R * R * math.asin(t / R))

    if y >= R:
        return 2.0 * (H(xe) - H(-R))
    w = math.sqrt(R * R - y * y)
    area = 0.0
    # inner part |X| <= w: y + h(X)
    a, b = -w, min(xe, w)
    if b > a:
        area += y * (b - a) + (H(b) - H(a))
    if y >= 0:
        # outer parts |X| > w: 2 h(X)
        a, b = -R, min(xe, -w)
        if b > a:
            area += 2.0 * (H(b) - H(a))
        a, b = w, xe
        if b > a:
            area += 2.0 * (H(b) - H(a))
    return area


def _rect_disk_area(x1, x2, y1, y2, R):
    return (_seg_area(x2, y2, R) - _seg_area(x1, y2, R)
            - _seg_area(x2, y1, R) + _seg_area(x1, y1, R))


def stencil_radius(rho, d):
    return int(math.ceil(rho / d + 0.5))


def disk_pixel_weights(rho, dx, dy):
    """FP64 weights [2Ry+1, 2Rx+1] (row = y offset); rho = 0 gives the identity."""
    if rho <= 0.0:
        return np.ones((1, 1))
    Rx = stencil_radius(rho, dx)
    Ry = stencil_radius(rho, dy)
    w = np.zeros((2 * Ry + 1, 2 * Rx + 1))
    for b in range(-Ry, Ry + 1):
        for a in range(-Rx, Rx + 1):
            # nearest / farthest point of the pixel from the disk centre
            nxd = max(0.0, (abs(a) - 0.5) * dx)
            nyd = max(0.0, (abs(b) - 0.5) * dy)
            fxd = (abs(a) + 0.5) * dx
            fyd = (abs(b) + 0.5) * dy
            if nxd * nxd + nyd * nyd >= rho * rho:
                area = 0.0  # pixel does not meet the disk
            elif fxd * fxd + fyd * fyd <= rho * rho:
                area = dx * dy  # pixel inside the disk
            else:
                area = _rect_disk_area((a - 0.5) * dx, (a + 0.5) * dx,
                                       (b - 0.5) * dy, (b + 0.5) * dy, rho)
            w[b + Ry, a + Rx] = area
    w /= math.pi * rho * rho
    w /= w.sum()
    # trim all-zero outer rings (they contribute nothing)
    while w.shape[0] > 1 and not w[0].any() and not w[-1].any():
        w = w[1:-1]
    while w.shape[1] > 1 and not w[:, 0].any() and not w[:, -1].any():
        w = w[:, 1:-1]
    return w


def map_scale(rays, window, fp32=True):
    """Normalisation factor (hx*hy)/(dx*dy); FP32 mirror uses binary32 spacings."""
    cx, cy, wx, wy, nx, ny = rays
    sx, sy, vx, vy, mx, my = window
    dx, dy = vx / mx, vy / my
    if fp32:
        hx = float(np.float32(wx / nx))
        hy = float(np.float32(wy / ny))
        return np.float32(hx * hy / (dx * dy))
    return (wx / nx) * (wy / ny) / (dx * dy)


def _shifted(c, db, da):
    """c[j+db, i+da] with edge clamping."""
    my, mx = c.shape
    jj = np.clip(np.arange(my) + db, 0, my - 1)
    ii = np.clip(np.arange(mx) + da, 0, mx - 1)
    return c[jj][:, ii]


def normalize_convolve_mirror32(counts, scale32, weights64):
    """Binary32 mirror: returns float32 [my, mx]."""
    w32 = np.asarray(weights64).astype(np.float32)
    c32 = np.asarray(counts).astype(np.float32)  # exact for counts <= 2^24
    Ry = (w32.shape[0] - 1) // 2
    Rx = (w32.shape[1] - 1) // 2
    acc = None
    for b in range(-Ry, Ry + 1):
        for a in range(-Rx, Rx + 1):
            wk = w32[b + Ry, a + Rx]
            if wk == 0:
                continue
            term = wk * _shifted(c32, b, a)
            acc = term if acc is None else acc + term
    return acc * np.float32(scale32)


def normalize_convolve_exact64(counts, scale64, weights64):
    c = np.asarray(counts).astype(np.float64)
    w = np.asarray(weights64)
    Ry = (w.shape[0] - 1) // 2
    Rx = (w.shape[1] - 1) // 2
    acc = np.zeros_like(c)
    for b in range(-Ry, Ry + 1):
        for a in range(-Rx, Rx + 1):
            if w[b + Ry, a + Rx] != 0:
                acc += w[b + Ry, a + Rx] * _shifted(c, b, a)
    return acc * scale64


def normalize_convolve_exact64_at(counts, scale64, weights64, pixels):
    """FP64 values at the listed (j, i) pixels only: sum over the stencil of
    w[b, a] * c[clamp(j + b), clamp(i + a)], times the scale (for wide stencils, where
    the whole-map version is too slow)."""
    c = np.asarray(counts)
    w = np.asarray(weights64, dtype=np.float64)
    my, mx = c.shape
    Ry = (w.shape[0] - 1) // 2
    Rx = (w.shape[1] - 1) // 2
    out = np.empty(len(pixels))
    for n, (j, i) in enumerate(pixels):
        jj = np.clip(np.arange(j - Ry, j + Ry + 1), 0, my - 1)
        ii = np.clip(np.arange(i - Rx, i + Rx + 1), 0, mx - 1)
        out[n] = float(np.sum(w * c[np.ix_(jj, ii)].astype(np.float64))) * scale64
    return out
