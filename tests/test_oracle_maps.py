"""Pins of oracle.maps: normalisation and uniform-disk convolution."""
import math

import numpy as np
import pytest

from oracle.maps import (_seg_area, disk_pixel_weights, map_scale,
                         normalize_convolve_exact64, normalize_convolve_mirror32)


def test_segment_area_special_cases():
    R = 0.7
    assert _seg_area(10, 10, R) == pytest.approx(math.pi * R * R, rel=1e-14)
    assert _seg_area(0, 10, R) == pytest.approx(math.pi * R * R / 2, rel=1e-14)
    assert _seg_area(0, 0, R) == pytest.approx(math.pi * R * R / 4, rel=1e-14)
    assert _seg_area(10, -R, R) == 0.0
    # a chord: {Y <= -R/2}: segment area R^2 (theta - sin theta)/2 with theta = 2 acos(1/2)
    th = 2 * math.acos(0.5)
    assert _seg_area(10, -R / 2, R) == pytest.approx(R * R * (th - math.sin(th)) / 2, rel=1e-13)


@pytest.mark.parametrize("rho,dx,dy", [(2e-3, 3 / 2048, 3 / 2048), (0.01, 3 / 1024, 3 / 1024),
                                       (0.004, 0.003, 0.002)])
def test_weights_match_supersampling(rho, dx, dy):
    w = disk_pixel_weights(rho, dx, dy)
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    Ry, Rx = (w.shape[0] - 1) // 2, (w.shape[1] - 1) // 2
    n = 1500
    xs = (np.arange(-(2 * Rx + 1) * n // 2, (2 * Rx + 1) * n // 2) + 0.5) * dx / n
    ys = (np.arange(-(2 * Ry + 1) * n // 2, (2 * Ry + 1) * n // 2) + 0.5) * dy / n
    X, Y = np.meshgrid(xs, ys)
    inside = X * X + Y * Y <= rho * rho
    ii = np.floor(X / dx + 0.5).astype(int) + Rx
    jj = np.floor(Y / dy + 0.5).astype(int) + Ry
    ws = np.zeros_like(w)
    np.add.at(ws, (jj[inside], ii[inside]), 1.0)
    ws /= inside.sum()
    assert np.abs(ws - w).max() < 2e-5
    assert np.allclose(w, w[::-1, :], atol=1e-15) and np.allclose(w, w[:, ::-1], atol=1e-15)


def test_small_disk_is_identity():
    assert np.array_equal(disk_pixel_weights(1e-3, 3 / 1024, 3 / 1024), np.ones((1, 1)))
    assert np.array_equal(disk_pixel_weights(0.0, 1.0, 1.0), np.ones((1, 1)))


def test_scale_is_ray_density_ratio():
    s32 = map_scale((0, 0, 4.0, 4.0, 3200, 3200), (0, 0, 2.0, 2.0, 512, 512))
    assert float(s32) == pytest.approx(0.1024, rel=1e-7)
    s64 = map_scale((0, 0, 6.0, 6.0, 32768, 32768), (0, 0, 3.0, 3.0, 2048, 2048), fp32=False)
    assert s64 == pytest.approx(1 / 64, rel=1e-15)


def test_constant_map_invariant_and_mirror_vs_exact():
    w = disk_pixel_weights(2e-3, 3 / 2048, 3 / 2048)
    c = np.full((64, 64), 64, dtype=np.uint32)
    A = normalize_convolve_mirror32(c, np.float32(1 / 64), w)
    assert np.abs(A - 1.0).max() < 1e-6
    rng = np.random.default_rng(0)
    c = rng.integers(0, 5000, (80, 96)).astype(np.uint32)
    A32 = normalize_convolve_mirror32(c, np.float32(1 / 64), w)
    A64 = normalize_convolve_exact64(c, 1 / 64, w)
    assert np.abs(A32 / A64 - 1)[A64 > 0].max() < 1e-6
    # brute-force one interior pixel
    j, i = 40, 50
    ref = sum(w[b + 1, a + 1] * float(c[j + b, i + a]) for b in (-1, 0, 1) for a in (-1, 0, 1)) / 64
    assert A64[j, i] == pytest.approx(ref, rel=1e-14)
    # edge clamp: corner pixel uses itself for outside neighbours
    ref = sum(w[b + 1, a + 1] * float(c[max(b, 0), max(a, 0)]) for b in (-1, 0, 1) for a in (-1, 0, 1)) / 64
    assert A64[0, 0] == pytest.approx(ref, rel=1e-14)


def test_per_pixel_sum_equals_whole_map_sum():
    from oracle.maps import normalize_convolve_exact64_at
    rng = np.random.default_rng(3)
    c = rng.integers(0, 5000, (40, 52)).astype(np.uint32)
    w = disk_pixel_weights(0.01, 3 / 1024, 3 / 1024)
    A = normalize_convolve_exact64(c, 1 / 64, w)
    px = [(0, 0), (39, 51), (0, 51), (39, 0), (20, 26), (3, 49)] + [(int(j), int(i)) for j, i in
                                                                   zip(rng.integers(0, 40, 30), rng.integers(0, 52, 30))]
    got = normalize_convolve_exact64_at(c, 1 / 64, w, px)
    ref = np.array([A[j, i] for j, i in px])
    assert np.allclose(got, ref, rtol=1e-13, atol=0)
