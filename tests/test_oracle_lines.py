"""Pins of oracle.lines: caustic-centred (r, phi) lines (sec. 4.2) and the
minimum-magnification filter (sec. 4.3)."""
import math

import numpy as np
import pytest

from oracle.lens import lens_setup, paczynski
from oracle.lines import (caustic_components, caustic_lines, line_filter_mirror32,
                          line_samples, lines_to_trajectories)
from oracle.sampling import trajectory_positions


@pytest.mark.parametrize("s,n", [(0.6, 3), (1.0, 1), (1.5, 1), (2.5, 2)])
def test_equal_mass_topology(s, n):
    # equal masses: close (three caustics) below s = 2^-1/2, intermediate (one) up to
    # s = 2, wide (two) above (the published transition separations)
    c = caustic_components(s, 1.0, 2048)
    assert len(c) == n


def test_symmetry_about_the_lens_axis():
    for s, q in ((0.6, 1.0), (0.5, 1e-3), (2.5, 0.3), (1.0, 0.1)):
        c = caustic_components(s, q, 2048)
        for cx, cy, hw, hh, size in c:
            if abs(cy) > 1e-9:  # off-axis caustics come in mirror pairs
                m = [v for v in c if abs(v[1] + cy) < 1e-9 and abs(v[0] - cx) < 1e-9]
                assert len(m) == 1 and abs(m[0][4] - size) < 1e-9 * max(size, 1e-12)
            assert size == max(hw, hh) and size > 0


def test_equal_mass_resonant_caustic_is_centred():
    (cx, cy, hw, hh, size), = caustic_components(1.0, 1.0, 4096)
    assert abs(cx) < 1e-12 and abs(cy) < 1e-12


def test_planetary_caustic_positions():
    q = 1e-4
    # wide: planetary caustic about s - 1/s from the host, on the axis
    s = 2.0
    m1, m2, x1, x2 = lens_setup(s, q)
    c = caustic_components(s, q, 8192)
    assert len(c) == 2
    host, planet = sorted(c, key=lambda v: v[0])
    assert planet[0] - x1 == pytest.approx(s - 1 / s, abs=1e-2)
    assert abs(planet[1]) < 1e-9
    # central caustic width along the axis about 4q/(s - 1/s)^2 (small-q limit)
    assert 2 * host[2] == pytest.approx(4 * q / (s - 1 / s) ** 2, rel=0.2)
    # close: two planetary caustics near x1 + s - 1/s, at +-2 sqrt(q)/(s sqrt(1 + s^2))
    s = 0.5
    m1, m2, x1, x2 = lens_setup(s, q)
    c = caustic_components(s, q, 8192)
    assert len(c) == 3
    lo, mid, hi = c  # ordered by cy
    assert lo[1] < -1e-3 and hi[1] > 1e-3 and abs(mid[1]) < 1e-9
    yp = 2 * math.sqrt(q) / (s * math.sqrt(1 + s * s))
    assert hi[1] == pytest.approx(yp, rel=0.2)
    assert hi[0] - x1 == pytest.approx(s - 1 / s, abs=0.05)


def test_lines_pass_at_r_sizes_from_the_caustic_centre():
    c = caustic_components(0.8, 5e-3, 2048)
    r = np.array([0.0, 0.5, 2.0])
    phi = np.array([0.3, 2.0, 4.5])
    L = caustic_lines(c, r, phi)
    assert L.shape == (len(c) * 9, 3)
    t0p, tE = 12.5, 20.0
    P = lines_to_trajectories(L, np.arange(len(L)), [t0p], [tE])
    for idx in range(len(L)):
        k, rest = divmod(idx, 9)
        j, l = divmod(rest, 3)
        cx, cy, _, _, size = c[k]
        z = trajectory_positions(P[idx], [t0p, t0p + tE])
        # at t0' the path is at the foot of the perpendicular from the caustic centre
        d = z[0] - (cx + 1j * cy)
        assert abs(d) == pytest.approx(r[j] * size, abs=1e-12)
        e = z[1] - z[0]  # one Einstein time later: moved by the unit direction e
        assert abs(e - complex(math.cos(phi[l]), math.sin(phi[l]))) < 1e-12
        assert abs((d.conjugate() * e).real) < 1e-12  # perpendicular


def test_line_samples_cover_the_window_at_pixel_spacing():
    win = (0.1, -0.2, 3.0, 2.0, 512, 256)
    tau, ns = line_samples(win, 0.7)
    assert ns == math.ceil(math.hypot(3.0, 2.0) * 512 / 3.0) + 1
    step = np.diff(tau.astype(np.float64))
    assert step.max() <= 3.0 / 512 * (1 + 1e-6)
    tc = 0.1 * math.cos(0.7) - 0.2 * math.sin(0.7)
    R = 0.5 * math.hypot(3.0, 2.0)
    assert tau[0] == pytest.approx(tc - R, abs=1e-6) and tau[-1] == pytest.approx(tc + R, abs=1e-5)


def test_filter_on_a_single_lens_map_reads_the_peak():
    # map filled with the single-lens magnification at pixel centres: the largest
    # sample along a line of impact u0 is the peak A(u0) (to bilinear/sampling error)
    nx = 512
    win = (0.0, 0.0, 2.0, 2.0, nx, nx)
    d = 2.0 / nx
    x = (np.arange(nx) - nx / 2 + 0.5) * d
    amap = paczynski(np.hypot(x[None, :], x[:, None])).astype(np.float32)
    u0s = np.array([0.05, 0.1, 0.3, 0.6])
    lines = np.stack([u0s, np.full(4, 0.4), np.zeros(4)], axis=1)
    best, keep = line_filter_mirror32(amap, win, lines, 2.0)
    assert np.allclose(best, paczynski(u0s), rtol=5e-3)
    assert list(keep) == list(paczynski(u0s) >= 2.0)
    # a line that misses the window keeps the off-map single-lens values: peak A(u0)
    far = np.array([[1.8, 0.0, 0.0]])
    b2, _ = line_filter_mirror32(amap, win, far, 1.0)
    assert b2[0] == pytest.approx(paczynski(1.8), rel=1e-6)


# ---- peak library and peak-time starts (sec. 4.3, third to fifth optimisations) ----
from oracle.lines import count_peaks, line_peaks_mirror32, peak_starts


def test_count_peaks_follows_the_gradient_sign_change():
    # a peak is where the gradient turns from positive to negative
    assert count_peaks([1, 2, 3, 2, 1]) == (1, [2])
    assert count_peaks([1, 2, 2, 2, 1]) == (1, [1])      # plateau: its first sample
    assert count_peaks([1, 3, 1, 3, 1]) == (2, [1, 3])
    assert count_peaks([3, 2, 1, 2]) == (0, [])          # maximum at the first sample
    assert count_peaks([1, 2, 3]) == (0, [])             # still rising at the end
    assert count_peaks([1, 2, 1, 2, 1, 2, 1], k_max=2) == (3, [1, 3])
    # hysteresis: wiggles within the relative band are not peaks
    assert count_peaks([1, 1.05, 1.0, 2, 1], h=0.1) == (1, [3])
    assert count_peaks([1, 1.05, 1.0, 2, 1], h=0.0) == (2, [1, 3])
    assert count_peaks([1, 2, 1.9, 2.1, 1], h=0.1) == (1, [3])


def _pixel_centres(n, V):
    c = -V / 2 + (np.arange(n) + 0.5) * V / n
    return np.meshgrid(c, c)


def test_single_lens_lines_have_one_peak_at_closest_approach():
    n, V = 256, 3.0
    X, Y = _pixel_centres(n, V)
    amap = paczynski(np.hypot(X, Y)).astype(np.float32)
    win = (0.0, 0.0, V, V, n, n)
    rng = np.random.default_rng(0)
    L = np.stack([rng.uniform(0.05, 0.8, 40), rng.uniform(0, 2 * np.pi, 40), np.zeros(40)], 1)
    tau, _ = line_samples(win, 0.0)
    spacing = float(tau[1] - tau[0])
    cnt, ptau, pA, best = line_peaks_mirror32(amap, win, L, h=0.0)
    assert np.all(cnt == 1)
    assert np.all(np.abs(ptau[:, 0]) <= 0.5 * spacing)   # M_p = 0: the closest approach
    assert np.array_equal(pA[:, 0], best)


@pytest.mark.parametrize("s,q", [(1.0, 1.0), (0.8, 0.2)])
def test_peaks_at_the_caustic_crossings(s, q):
    """On a smooth point-source map (quintic magnification at pixel centres) a horizontal
    line has a peak within 1.5 pixels of each place where it crosses the caustic."""
    from oracle.caustics import caustic_points
    from oracle.lens import point_source_magnification
    n, V = 256, 3.0
    X, Y = _pixel_centres(n, V)
    amap = point_source_magnification((X + 1j * Y).ravel(), s, q).reshape(n, n).astype(np.float32)
    win = (0.0, 0.0, V, V, n, n)
    z = np.asarray(caustic_points(s, q, 8192)).reshape(-1)
    for u0 in (0.03, 0.1, -0.07):
        cnt, ptau, _, _ = line_peaks_mirror32(amap, win, np.array([[u0, 0.0, 0.0]]), h=0.05)
        xs = np.sort(z[np.abs(z.imag - u0) < 2e-3].real)
        groups = np.split(xs, np.flatnonzero(np.diff(xs) > 0.02) + 1)
        crossings = [g.mean() for g in groups if len(g)]
        assert len(crossings) >= 2
        peaks = ptau[0, :cnt[0]]
        for x in crossings:
            assert np.min(np.abs(peaks - x)) < 1.5 * V / n, (u0, x, peaks)


def test_peak_times_recover_t0_and_tE():
    """Eqs. 7-8: peaks observed at t_pi = t0 + M_pi tE give back (t0, tE) of each line."""
    rng = np.random.default_rng(3)
    n, K = 30, 8
    lines = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(0, 2 * np.pi, n),
                      rng.uniform(-1, 1, n)], 1)
    cnt = rng.integers(2, 6, n).astype(np.int32)
    ptau = np.full((n, K), np.nan, np.float32)
    pA = np.full((n, K), np.nan, np.float32)
    for i in range(n):
        ptau[i, :cnt[i]] = np.sort(rng.uniform(-1.5, 1.5, cnt[i])).astype(np.float32)
        pA[i, :cnt[i]] = rng.uniform(1.5, 30.0, cnt[i]).astype(np.float32)
    t0, tE = 2456123.4, 23.5
    for i in range(n):
        top = sorted(np.argsort(-pA[i, :cnt[i]])[:2])
        m1, m2 = float(ptau[i, top[0]]), float(ptau[i, top[1]])
        tp = [t0 + m1 * tE, t0 + m2 * tE]
        st = peak_starts(lines[i:i + 1], cnt[i:i + 1], ptau[i:i + 1], pA[i:i + 1], tp)[0]
        assert abs(st[1] - tE) < 1e-9 * tE
        assert abs((st[0] - lines[i, 2] * st[1]) - t0) < 1e-6     # t0 = t0' - shift tE
        # one observed peak: the highest, with tE given (Eq. 7)
        hi = int(np.argmax(pA[i, :cnt[i]]))
        st1 = peak_starts(lines[i:i + 1], cnt[i:i + 1], ptau[i:i + 1], pA[i:i + 1],
                          [t0 + float(ptau[i, hi]) * tE], tE_default=tE)[0]
        assert abs((st1[0] - lines[i, 2] * tE) - t0) < 1e-6 and st1[1] == tE
    # a line with fewer peaks than observed times gets no start
    one = np.array([1], np.int32)
    assert np.isnan(peak_starts(lines[:1], one, ptau[:1], pA[:1], [1.0, 2.0])).all()
