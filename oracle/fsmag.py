"""Image-centred ray-shooting finite-source magnification (test infrastructure only).

Sec. 5 refines solutions without maps: for a trial (d, q) it finds the caustics, uses
the point-source magnification when the source lies more than 10 rho from the nearest
caustic, and otherwise shoots rays around the source's images: the images of points on
the source boundary and its centre are found, a polar grid about each image is grown
until it holds the whole image, and the source intensity at each grid point, found by
inverse ray shooting through Eq. 2, is integrated over the images with a second-order
treatment of the source boundary.  The paper gives no further detail; the readings
fixed here (and mirrored, in its own code, by the GPU) are:

  * proximity: the distance from the source centre to the nearest of the caustic
    points (Eq. 2 images of the critical-curve points at n_crit phases); > 10 rho ->
    point-source magnification of the centre's images (Eqs. 3-4).
  * seeds: the images of the centre and of n_b boundary points zeta_s + rho
    exp(2 pi i (j + 1/2)/n_b), and the critical points whose caustic image lies inside
    the source (where a grazing source creates images the boundary samples may miss):
    of those at phases p with p mod m = 0, m the smallest stride >= ceil(count / 512)
    that keeps at most 512; in polar coordinates (r, theta) about the centre of mass.
  * regions: seeds sorted by theta; the circle is cut at every gap wider than
    ``gap`` (0.2 rad); each run of seeds is a region [r_min, r_max] x [theta_a,
    theta_b] (a full ring when no gap is wider), padded by 10 % of its extent plus
    rho in r and rho / r_max in theta.
    Within a run, the seeds sorted by r are split where consecutive radii differ by
    more than max(gap r, 4 rho).
  * growth: each side of a region is sampled at n_side points (corners included); a
    side on which any sample maps inside the source (|zeta(z) - zeta_s| < rho) moves
    out by a quarter of the region's extent in that coordinate (r >= 0; a theta extent
    reaching 2 pi makes a ring); repeated until no side moves (at most ``n_grow``
    rounds).  Then overlapping regions are replaced by their union until none overlap.
  * shrink: after integrating a region it is cut to the radial nodes and columns that
    hold inside nodes, one cell wider on each side, and integrated again (at most
    n_shrink = 2 times), so the grid follows the image's own extent.
  * integral: each region is cut into n_theta columns (midpoints) of n_r radial
    segments; along a column, f = rho^2 - |zeta(z) - zeta_s|^2 at the nodes marks the
    inside (f > 0) and is taken linear along each segment, so a segment crossing the
    limb keeps its inside part up to r* = r_a + dr f_a/(f_a - f_b).  With the
    limb-darkened profile in its Gamma form with unit mean over the disk,
    I = 1 - Gamma + 1.5 Gamma sqrt(f)/rho, the inside part [lo, hi] of a segment adds
    r_m (hi - lo) [(1 - Gamma) + (1.5 Gamma/rho) (2/3)(a^2 + ab + b^2)/(a + b)],
    r_m its midpoint and a, b the square roots of f at its ends (0 at the limb): the
    mean of sqrt(f) for f linear, so the square-root edge of the profile is integrated
    exactly (second order overall).  Columns add with d theta; the magnification is
    the integral over pi rho^2.
All arithmetic is FP64.
"""
from __future__ import annotations

import math

import numpy as np

from .caustics import critical_curve_points
from .lens import image_positions, lens_equation, point_source_magnification

__all__ = ["FsOptions", "critical_points_and_caustic", "fs_magnification", "regions_of",
           "single_lens_disk", "brute_force_fs"]


class FsOptions:
    def __init__(self, n_b=192, n_crit=1024, near=10.0, gap=0.2, n_side=128, n_grow=40,
                 n_r=512, n_theta=512, n_shrink=2):
        self.n_b, self.n_crit, self.near, self.gap = n_b, n_crit, near, gap
        self.n_side, self.n_grow, self.n_r, self.n_theta = n_side, n_grow, n_r, n_theta
        self.n_shrink = n_shrink


def critical_points_and_caustic(s, q, n_crit):
    z = critical_curve_points(s, q, n_crit).reshape(-1)
    return z, lens_equation(z, s, q)


def _profile(x, gamma):
    return 1.0 - gamma * (1.0 - 1.5 * np.sqrt(np.maximum(1.0 - x, 0.0)))


def _inside(z, zeta_s, rho, s, q):
    return np.abs(lens_equation(z, s, q) - zeta_s) < rho


CRIT_SEEDS = 512  # critical-point seeds at most


def _seeds(zeta_s, rho, s, q, zc, cc, opt):
    pts = [zeta_s] + list(zeta_s + rho * np.exp(2j * np.pi * (np.arange(opt.n_b) + 0.5) / opt.n_b))
    roots, isimg = image_positions(np.array(pts), s, q)
    z = roots[isimg]
    inside = np.abs(cc - zeta_s) < rho
    phase = np.arange(len(cc)) // 4
    m = max(1, -(-int(inside.sum()) // CRIT_SEEDS))
    while int((inside & (phase % m == 0)).sum()) > CRIT_SEEDS:
        m += 1
    z = np.concatenate([z, zc[inside & (phase % m == 0)]])
    return z


def regions_of(z, rho, opt):
    """Initial polar regions [(r0, r1, t0, t1)] (t1 - t0 = 2 pi: a ring) of seeds z."""
    r = np.abs(z)
    th = np.angle(z)
    o = np.argsort(th, kind="stable")
    r, th = r[o], th[o]
    gaps = np.diff(np.append(th, th[0] + 2 * np.pi))
    cut = np.flatnonzero(gaps > opt.gap)
    out = []
    if len(cut) == 0:
        out.append([float(r.min()), float(r.max()), -math.pi, math.pi])
    else:
        n = len(th)
        for a, b in zip(cut, np.roll(cut, -1)):
            idx = [(a + 1 + k) % n for k in range(((b - a - 1) % n) + 1)]
            t = th[idx].copy()
            t[t < t[0]] += 2 * np.pi  # unwrap across +-pi
            rr = r[idx]
            # split the angular run where its seeds' radii leave a gap
            o2 = np.argsort(rr, kind="stable")
            rs, ts = rr[o2], t[o2]
            cuts = np.flatnonzero(np.diff(rs) > np.maximum(opt.gap * rs[1:], 4.0 * rho)) + 1
            for part in np.split(np.arange(len(rs)), cuts):
                out.append([float(rs[part].min()), float(rs[part].max()), float(ts[part].min()),
                            float(ts[part].max())])
    regs = []
    for r0, r1, t0, t1 in out:
        dr = 0.1 * (r1 - r0) + rho
        r0, r1 = max(0.0, r0 - dr), r1 + dr
        if t1 - t0 < 2 * np.pi:
            dt = 0.1 * (t1 - t0) + rho / max(r1, 1e-12)
            t0, t1 = t0 - dt, t1 + dt
        if t1 - t0 >= 2 * np.pi:
            t0, t1 = -math.pi, math.pi
        regs.append([r0, r1, t0, t1])
    return regs


def _ring(reg):
    return reg[3] - reg[2] >= 2 * np.pi


def _side_hits(reg, zeta_s, rho, s, q, n):
    """Whether any sample of each side (r0, r1, t0, t1) maps inside the source."""
    r0, r1, t0, t1 = reg
    tt = np.linspace(t0, t1, n)
    rr = np.linspace(r0, r1, n)
    hits = [bool(_inside(r0 * np.exp(1j * tt), zeta_s, rho, s, q).any()),
            bool(_inside(r1 * np.exp(1j * tt), zeta_s, rho, s, q).any())]
    if _ring(reg):
        hits += [False, False]
    else:
        hits += [bool(_inside(rr * np.exp(1j * t0), zeta_s, rho, s, q).any()),
                 bool(_inside(rr * np.exp(1j * t1), zeta_s, rho, s, q).any())]
    return hits


def _grow(reg, zeta_s, rho, s, q, opt):
    reg = list(reg)
    for _ in range(opt.n_grow):
        h = _side_hits(reg, zeta_s, rho, s, q, opt.n_side)
        if not any(h):
            break
        dr = 0.25 * (reg[1] - reg[0])
        dt = 0.25 * (reg[3] - reg[2])
        if h[0]:
            reg[0] = max(0.0, reg[0] - dr)
        if h[1]:
            reg[1] = reg[1] + dr
        if h[2]:
            reg[2] = reg[2] - dt
        if h[3]:
            reg[3] = reg[3] + dt
        if reg[3] - reg[2] >= 2 * np.pi:
            reg[2], reg[3] = -math.pi, math.pi
    return reg


def _theta_overlap(a, b):
    if _ring(a) or _ring(b):
        return True
    # shift b by multiples of 2 pi to the copy nearest a
    k = round(((a[2] + a[3]) - (b[2] + b[3])) / (4 * np.pi))
    b2, b3 = b[2] + 2 * np.pi * k, b[3] + 2 * np.pi * k
    return not (b3 < a[2] or b2 > a[3])


def _union(a, b):
    r0, r1 = min(a[0], b[0]), max(a[1], b[1])
    if _ring(a) or _ring(b):
        return [r0, r1, -math.pi, math.pi]
    k = round(((a[2] + a[3]) - (b[2] + b[3])) / (4 * np.pi))
    t0, t1 = min(a[2], b[2] + 2 * np.pi * k), max(a[3], b[3] + 2 * np.pi * k)
    if t1 - t0 >= 2 * np.pi:
        t0, t1 = -math.pi, math.pi
    return [r0, r1, t0, t1]


def _merge(regs):
    regs = [list(r) for r in regs]
    changed = True
    while changed:
        changed = False
        for i in range(len(regs)):
            for j in range(i + 1, len(regs)):
                a, b = regs[i], regs[j]
                if not (b[1] < a[0] or b[0] > a[1]) and _theta_overlap(a, b):
                    regs[i] = _union(a, b)
                    del regs[j]
                    changed = True
                    break
            if changed:
                break
    return regs


def _integrate(reg, zeta_s, rho, gamma, s, q, opt):
    r0, r1, t0, t1 = reg
    dth = (t1 - t0) / opt.n_theta
    th = t0 + (np.arange(opt.n_theta) + 0.5) * dth
    dr = (r1 - r0) / opt.n_r
    r = r0 + np.arange(opt.n_r + 1) * dr
    z = r[None, :] * np.exp(1j * th)[:, None]
    f = rho * rho - np.abs(lens_equation(z, s, q) - zeta_s) ** 2
    fa, fb = f[:, :-1], f[:, 1:]
    ra = np.broadcast_to(r[None, :-1], fa.shape)
    rb = ra + dr
    with np.errstate(invalid="ignore", divide="ignore"):
        rs = ra + dr * fa / (fa - fb)            # the limb, f linear along the segment
    ina, inb = fa > 0, fb > 0
    lo = np.where(ina, ra, np.where(inb, rs, 0.0))  # inside part [lo, hi] of the segment
    hi = np.where(inb, rb, np.where(ina, rs, 0.0))
    sa = np.sqrt(np.where(ina, fa, 0.0))
    sb = np.sqrt(np.where(inb, fb, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        mean_sqrt = np.where(sa + sb > 0, (2.0 / 3.0) * (sa * sa + sa * sb + sb * sb) / (sa + sb), 0.0)
    L = hi - lo
    rm = 0.5 * (lo + hi)
    seg = (1.0 - gamma) * rm * L + (1.5 * gamma / rho) * rm * L * mean_sqrt
    seg = np.where(ina | inb, seg, 0.0)
    inside = f > 0
    cols = np.flatnonzero(inside.any(axis=1))
    rows = np.flatnonzero(inside.any(axis=0))
    box = (int(rows[0]), int(rows[-1]), int(cols[0]), int(cols[-1])) if len(cols) else None
    return float(seg.sum()) * dth, box


def _shrink(reg, box, opt):
    """The region cut to the nodes and columns holding inside nodes, one cell wider."""
    r0, r1, t0, t1 = reg
    if box is None:
        return None
    k0, k1, j0, j1 = box
    dr = (r1 - r0) / opt.n_r
    n0, n1 = max(k0 - 1, 0), min(k1 + 1, opt.n_r)
    out = [r0 + n0 * dr, r0 + n1 * dr, t0, t1]
    if not _ring(reg):
        dth = (t1 - t0) / opt.n_theta
        out[2] = t0 + max(j0 - 1, 0) * dth
        out[3] = t0 + min(j1 + 2, opt.n_theta) * dth
    return out


def fs_magnification(zeta_s, rho, gamma, s, q, opt=None, crit=None, details=False):
    """Finite-source magnification of a source at zeta_s (complex) of radius rho."""
    opt = opt or FsOptions()
    zc, cc = crit if crit is not None else critical_points_and_caustic(s, q, opt.n_crit)
    zeta_s = complex(zeta_s)
    dist = float(np.nanmin(np.abs(cc - zeta_s)))
    if dist > opt.near * rho:
        A = float(point_source_magnification(np.array([zeta_s]), s, q)[0])
        return (A, {"point_source": True, "regions": []}) if details else A
    seeds = _seeds(zeta_s, rho, s, q, zc, cc, opt)
    regs = [_grow(r, zeta_s, rho, s, q, opt) for r in regions_of(seeds, rho, opt)]
    regs = _merge(regs)
    total = 0.0
    final = []
    for reg in regs:
        # integrate; cut the region to its inside cells (one cell wider) and integrate
        # again, at most n_shrink times
        val, box = _integrate(reg, zeta_s, rho, gamma, s, q, opt)
        for _ in range(opt.n_shrink):
            nxt = _shrink(reg, box, opt)
            if nxt is None or nxt == reg:
                break
            reg = nxt
            val, box = _integrate(reg, zeta_s, rho, gamma, s, q, opt)
        total += val
        final.append(reg)
    regs = final
    A = total / (math.pi * rho * rho)
    return (A, {"point_source": False, "regions": regs}) if details else A


# ---------------------------------------------------------------- references (pins)
def single_lens_disk(b, rho, gamma=0.0, n=400):
    """Finite-source magnification of a point lens at the origin, source centre at
    distance b, by polar integration about the lens: A = (1/(pi rho^2)) int dphi
    int_{u1}^{u2} I A_ps(u) u du.  Uniform disk (gamma = 0): the inner integral is exact,
    (1/2)[u sqrt(u^2 + 4)], so one Gauss-Legendre sum over phi remains; limb-darkened:
    Gauss-Legendre in u as well.  The lens inside the source (b < rho) has u1 = 0."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    if b < rho:
        phi = math.pi * (xg + 1.0)            # [0, 2 pi]
        wphi = math.pi * wg
    else:
        pm = math.asin(min(1.0, rho / b))
        phi = pm * xg                          # the source subtends [-pm, pm]
        wphi = pm * wg
    c = b * np.cos(phi)
    disc = np.sqrt(np.maximum(rho * rho - (b * np.sin(phi)) ** 2, 0.0))
    u2 = c + disc
    u1 = np.maximum(c - disc, 0.0) if b >= rho else np.zeros_like(c)
    if gamma == 0.0:
        F = lambda u: 0.5 * u * np.sqrt(u * u + 4.0)
        inner = F(u2) - F(u1)
    else:
        x = 0.5 * (xg + 1.0)
        wx = 0.5 * wg
        u = u1[:, None] + (u2 - u1)[:, None] * x[None, :]
        d2 = u * u + b * b - 2.0 * u * b * np.cos(phi)[:, None]
        I = _profile(d2 / (rho * rho), gamma)
        Au = (u * u + 2.0) / np.sqrt(u * u + 4.0)  # A(u) u
        inner = ((I * Au) @ wx) * (u2 - u1)
    return float(inner @ wphi) / (math.pi * rho * rho)


def brute_force_fs(zeta_s, rho, gamma, s, q, box, n, chunk=2048):
    """Uniform inverse ray shooting over the square image-plane box (cx, cy, half-side)
    with n x n rays at cell centres: sum of I over the rays landing in the source times
    the cell area, over pi rho^2.  Converges like the cell size (no boundary
    treatment); a plain check on the whole image plane."""
    cx, cy, hw = box
    h = 2.0 * hw / n
    xs = cx - hw + (np.arange(n) + 0.5) * h
    tot = 0.0
    for a in range(0, n, chunk):
        ys = cy - hw + (np.arange(a, min(a + chunk, n)) + 0.5) * h
        z = xs[None, :] + 1j * ys[:, None]
        d2 = np.abs(lens_equation(z, s, q) - zeta_s) ** 2
        inside = d2 < rho * rho
        tot += float(np.where(inside, _profile(d2 / (rho * rho), gamma), 0.0).sum())
    return tot * h * h / (math.pi * rho * rho)
