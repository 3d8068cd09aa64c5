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
