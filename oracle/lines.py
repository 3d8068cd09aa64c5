"""Caustic-centred trajectory lines and the minimum-magnification filter (test
infrastructure only).

Sec. 4.2 replaces the search over the impact parameter u0 about the lens centre by a
search over radial distances r from the centres of the caustics, scaled by the caustic
sizes, and angles phi (Fig. 1: one (r, phi) search space per caustic).  Sec. 4.3
(first optimisation) discards a trajectory whose magnification along its path, read
from the point-source map, never reaches the minimum magnification the light curve
implies.

Readings fixed here (the paper gives none of these details):
  * caustics: the quartic critical-curve equation (see ``caustics``) is solved at nphi
    equally spaced phases; each critical point is joined to the nearest critical point
    of the next phase (cyclically), and the connected sets are the separate critical
    curves.  Each one's caustic (Eq. 2 image of its points) has a bounding box; its
    centre is the box centre and its size the larger half-side.  Caustics are listed by
    (round(1e9 cy), cx) ascending.
  * lines: caustic k, radial distance r (in units of its size) and angle phi give the
    straight path zeta(tau) = c_k + r S_k n + tau e, e = (cos phi, sin phi),
    n = (-sin phi, cos phi).  In the (u0, alpha) form zeta = tau' e + u0 n it is
    alpha = phi, u0 = r S_k - cx sin phi + cy cos phi, with tau' = tau + shift,
    shift = cx cos phi + cy sin phi.  Lines are ordered caustic, then r, then phi.
  * trajectories of a line: for a time of closest approach to the caustic centre t0'
    and Einstein time tE, t0 = t0' - shift tE (same u0, tE, alpha); ordered line, then
    t0', then tE.
  * peaks (sec. 4.3, third optimisation): a peak is where the magnification along the
    line stops rising and starts falling.  On the filter's binary32 samples A_k, in
    order of tau, with relative hysteresis h >= 0 (so that the counting noise of a
    ray-shooting map does not make peaks; h = 0 is the literal definition): after a
    trough m (initially the first sample), a rise is a sample a > fl32(m fl32(1 + h));
    after a rise, the running maximum M (first sample of equal maxima) becomes a peak
    when a sample a < fl32(M fl32(1 - h)) follows, and that sample starts the next
    trough.  A maximum at the first sample or one still rising at the last is no peak.
    The library keeps the count and the positions tau (from the t0 point, the M_p of
    Eqs. 7-8) and values of the first K peaks.
  * starts (sec. 4.3, fourth and fifth optimisations): with one observed peak time t_p
    and a given tE, the line's highest peak M_p gives t0 = t_p - M_p tE (Eq. 7); with two
    observed times t_p1 < t_p2 its two highest peaks, in tau order M_1 < M_2, give
    tE = (t_p2 - t_p1)/(M_2 - M_1) (Eq. 8) and t0 = t_p1 - M_1 tE.  The simplex start is
    (t0' = t0 + shift tE, tE); a line with fewer peaks than observed times gets NaN.
  * filter: the line is sampled across the map window, over tau' in
    [tau_c - R, tau_c + R] with tau_c = cxw cos phi + cyw sin phi (window centre) and R
    half the window diagonal, at n_s = ceil(2 R kmax) + 1 points (kmax = the larger of
    M/V: at most one pixel apart): tau_k = fl32(tau_c - R) + k fl32(2R/(n_s - 1)) in
    binary32, sampled exactly as the search samples a point (binary32 geometry,
    bilinear on the map, single-lens value off it) with t0' = 0 and 1/tE = 1.  The line
    is kept when the largest sample is >= fl32(A_min).
"""
from __future__ import annotations

import math

import numpy as np

from .caustics import critical_curve_points
from .lens import lens_equation
from .sampling import sample_mirror32

__all__ = ["caustic_components", "caustic_lines", "line_filter_mirror32", "line_samples",
           "lines_to_trajectories", "count_peaks", "line_peaks_mirror32", "peak_starts"]

_f = np.float32


def _components(z):
    """Connected sets of critical points [nphi, 4] linked to their nearest point of the
    next phase; returns a label per point (labels in order of first appearance)."""
    nphi, nr = z.shape
    parent = list(range(nphi * nr))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    nxt = np.roll(z, -1, axis=0)
    d = np.abs(nxt[:, None, :] - z[:, :, None])  # [p, k, k']
    link = np.argmin(d, axis=2)
    for p in range(nphi):
        for k in range(nr):
            a = find(p * nr + k)
            b = find(((p + 1) % nphi) * nr + int(link[p, k]))
            if a != b:
                parent[max(a, b)] = min(a, b)
    roots = np.array([find(i) for i in range(nphi * nr)]).reshape(nphi, nr)
    return roots


def caustic_components(s: float, q: float, nphi: int = 4096):
    """[n, 5] array of (cx, cy, half_w, half_h, size) per separate caustic."""
    z = critical_curve_points(s, q, nphi)
    lab = _components(z)
    zeta = lens_equation(z, s, q)
    out = []
    for r in np.unique(lab):
        c = zeta[lab == r]
        x0, x1 = c.real.min(), c.real.max()
        y0, y1 = c.imag.min(), c.imag.max()
        hw, hh = 0.5 * (x1 - x0), 0.5 * (y1 - y0)
        out.append((0.5 * (x0 + x1), 0.5 * (y0 + y1), hw, hh, max(hw, hh)))
    out.sort(key=lambda v: (round(v[1] * 1e9), v[0]))
    return np.array(out, dtype=np.float64).reshape(-1, 5)


def caustic_lines(caustics, r, phi):
    """[n_caustics * n_r * n_phi, 3] lines (u0, alpha, shift)."""
    cs = np.asarray(caustics, dtype=np.float64).reshape(-1, 5)
    out = []
    for cx, cy, _, _, size in cs:
        for rv in np.asarray(r, dtype=np.float64):
            for ph in np.asarray(phi, dtype=np.float64):
                sn, cn = math.sin(ph), math.cos(ph)
                u0 = rv * size - cx * sn + cy * cn
                shift = cx * cn + cy * sn
                out.append((u0, ph, shift))
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def lines_to_trajectories(lines, kept, t0, tE):
    """[len(kept) * n_t0 * n_tE, 4] FP64 (t0, u0, tE, alpha)."""
    L = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    out = []
    for ell in kept:
        u0, al, shift = L[int(ell)]
        for a in np.asarray(t0, dtype=np.float64):
            for b in np.asarray(tE, dtype=np.float64):
                out.append((a - shift * b, u0, b, al))
    return np.array(out, dtype=np.float64).reshape(-1, 4)


def line_samples(window, alpha):
    """Binary32 sample positions tau_k [n_s] along a line of angle alpha, and n_s."""
    cxw, cyw, vx, vy, mx, my = window
    R = 0.5 * math.sqrt(vx * vx + vy * vy)
    kmax = max(mx / vx, my / vy)
    ns = int(math.ceil(2.0 * R * kmax)) + 1
    tau_c = cxw * math.cos(alpha) + cyw * math.sin(alpha)
    lo = _f(tau_c - R)
    h = _f(2.0 * R / (ns - 1))
    k = np.arange(ns, dtype=np.float32)
    return lo + k * h, ns


def line_filter_mirror32(amap, window, lines, a_min):
    """Largest binary32 sample along each line (float32 [n]) and keep flags (bool [n])."""
    L = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    best = np.empty(len(L), dtype=np.float32)
    for i, (u0, al, _) in enumerate(L):
        tau, _ = line_samples(window, al)
        sn, cn = math.sin(al), math.cos(al)
        consts = dict(t0p=np.array([0.0], _f), iE=np.array([1.0], _f), ca=np.array([cn], _f),
                      sa=np.array([sn], _f), bx=np.array([-u0 * sn], _f), by=np.array([u0 * cn], _f))
        best[i] = sample_mirror32(amap, window, consts, tau)[0].max()
    return best, best >= _f(a_min)


def count_peaks(a, h=0.0, k_max=8):
    """Peaks of the sequence a (float32) with relative hysteresis h: (count, indices of
    the first k_max peaks).  Pure-Python scan of the rule above."""
    a = np.asarray(a, dtype=np.float32)
    up, down = _f(1.0 + h), _f(1.0 - h)
    count, idx = 0, []
    trough = a[0]
    rising = False
    top, top_i = a[0], 0
    for i in range(1, len(a)):
        v = a[i]
        if not rising:
            if v < trough:
                trough = v
            elif v > _f(trough * up):
                rising, top, top_i = True, v, i
        else:
            if v > top:
                top, top_i = v, i
            elif v < _f(top * down):
                if count < k_max:
                    idx.append(top_i)
                count += 1
                rising, trough = False, v
    return count, idx


def line_peaks_mirror32(amap, window, lines, h=0.0, k_max=8):
    """Peak library of each line on the binary32 samples of the filter: count [n] int,
    positions tau [n, k_max] float32 and values A [n, k_max] float32 (NaN past the
    count), and the largest sample [n] float32."""
    L = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    n = len(L)
    cnt = np.zeros(n, dtype=np.int32)
    ptau = np.full((n, k_max), np.nan, dtype=np.float32)
    pA = np.full((n, k_max), np.nan, dtype=np.float32)
    best = np.empty(n, dtype=np.float32)
    for i, (u0, al, _) in enumerate(L):
        tau, _ = line_samples(window, al)
        sn, cn = math.sin(al), math.cos(al)
        consts = dict(t0p=np.array([0.0], _f), iE=np.array([1.0], _f), ca=np.array([cn], _f),
                      sa=np.array([sn], _f), bx=np.array([-u0 * sn], _f), by=np.array([u0 * cn], _f))
        A = sample_mirror32(amap, window, consts, tau)[0]
        best[i] = A.max()
        cnt[i], idx = count_peaks(A, h, k_max)
        ptau[i, :len(idx)] = tau[idx]
        pA[i, :len(idx)] = A[idx]
    return cnt, ptau, pA, best


def peak_starts(lines, count, ptau, pA, tp, tE_default=None):
    """Simplex starts (t0', tE) [n, 2] FP64 from observed peak times tp (one or two,
    ascending) by Eqs. 7-8 on each line's highest peaks; NaN rows for lines with fewer
    peaks than observed times."""
    L = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    tp = [float(v) for v in np.atleast_1d(tp)]
    out = np.full((len(L), 2), np.nan)
    for i in range(len(L)):
        k = min(int(count[i]), ptau.shape[1])
        if k < len(tp):
            continue
        vals = [float(v) for v in pA[i, :k]]
        # highest first; equal heights: the earlier peak first
        order = sorted(range(k), key=lambda j: (-vals[j], j))
        shift = L[i, 2]
        if len(tp) == 1:
            tE = float(tE_default)
            t0 = tp[0] - float(ptau[i, order[0]]) * tE
        else:
            j1, j2 = sorted(order[:2])
            m1, m2 = float(ptau[i, j1]), float(ptau[i, j2])
            tE = (tp[1] - tp[0]) / (m2 - m1)
            t0 = tp[0] - m1 * tE
        out[i] = (t0 + shift * tE, tE)
    return out
