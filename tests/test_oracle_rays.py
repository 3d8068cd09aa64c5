"""Pins of oracle.rays: the ray-count histogram (Eq. 2 ray shooting)."""
import numpy as np
import pytest

import workloads as W
from oracle.caustics import caustic_mask
from oracle.lens import point_source_magnification, paczynski
from oracle.maps import map_scale
from oracle.rays import (ray_positions_mirror32, rayshoot_exact64, rayshoot_mirror32_c,
                         rayshoot_mirror32_numpy)

TINY = W.config("tiny")


def test_c_and_numpy_mirrors_bit_exact_tiny():
    c = TINY
    cc, sc = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=4)
    cn, sn = rayshoot_mirror32_numpy(c["s"], c["q"], c["rays"], c["window"])
    assert np.array_equal(cc, cn)
    assert sc == sn


@pytest.mark.parametrize("s,q,rays,window", [
    (0.8, 5e-3, (0.1, -0.05, 3.0, 2.5, 640, 512), (0.02, 0.01, 1.5, 1.2, 200, 160)),
    (2.0, 0.3, (0.0, 0.0, 6.0, 6.0, 1024, 1024), (0.5, 0.0, 3.0, 3.0, 256, 256)),
])
def test_c_and_numpy_mirrors_bit_exact_offcentre(s, q, rays, window):
    cc, sc = rayshoot_mirror32_c(s, q, rays, window, nthreads=3)
    cn, sn = rayshoot_mirror32_numpy(s, q, rays, window)
    assert np.array_equal(cc, cn)
    assert sc == sn


def test_conservation_and_mirror_symmetry():
    c = TINY
    cnt, st = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=4)
    n = c["rays"][4] * c["rays"][5]
    assert int(cnt.sum(dtype=np.uint64)) + st["out"] + st["nonfinite"] == n
    assert st["zero_axis"] == 0
    # symmetric lattice and bin rule -> exact mirror symmetry about the lens axis
    assert np.array_equal(cnt, cnt[::-1, :])


def test_row_ranges_accumulate():
    c = TINY
    full, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"])
    part = np.zeros_like(full)
    for a, b in [(0, 1000), (1000, 1001), (1001, 3200)]:
        rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], rows=(a, b), counts=part)
    assert np.array_equal(full, part)


def test_fp32_vs_fp64_bins_rarely_differ():
    c = TINY
    c32, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=4)
    c64, _ = rayshoot_exact64(c["s"], c["q"], c["rays"], c["window"])
    rel_l1 = np.abs(c64.astype(np.int64) - c32.astype(np.int64)).sum() / c64.sum()
    assert rel_l1 < 1e-3


def test_single_lens_annulus_closed_form():
    # q = 0: the rays with |zeta| < R come from the annulus r+- = (+-R + sqrt(R^2+4))/2
    # of area pi R sqrt(R^2+4), i.e. that many rays per unit lattice cell area.
    rays = (0.0, 0.0, 5.0, 5.0, 2000, 2000)
    window = (0.0, 0.0, 2.0, 2.0, 64, 64)
    zx, zy, _, _ = ray_positions_mirror32(1.0, 0.0, rays, window, (0, 2000))
    h = 5.0 / 2000
    r = np.hypot(zx.astype(np.float64), zy.astype(np.float64))
    for R in (0.1, 0.5, 1.0):
        expect = np.pi * R * np.sqrt(R * R + 4) / (h * h)
        assert np.count_nonzero(r < R) == pytest.approx(expect, rel=1e-3)


def test_single_lens_map_matches_paczynski_blocks():
    rays = (0.0, 0.0, 4.0, 4.0, 3200, 3200)
    window = (0.0, 0.0, 2.0, 2.0, 512, 512)
    cnt, _ = rayshoot_mirror32_c(1.0, 0.0, rays, window, nthreads=4)
    A = cnt.astype(np.float64) * float(map_scale(rays, window))
    B = 16
    Ab = A.reshape(32, B, 32, B).mean(axis=(1, 3))
    d = 2.0 / 512
    sub = (np.arange(4 * B) + 0.5) / (4 * B) * B * d  # 64 x 64 samples per block
    cx = -1.0 + np.arange(32) * B * d
    X = cx[:, None] + sub[None, :]
    truth = np.zeros((32, 32))
    for j in range(32):
        U = np.hypot(X[:, :, None], X[j][None, None, :])
        truth[j] = paczynski(U).mean(axis=(1, 2))
    ok = np.ones((32, 32), bool)
    ok[14:18, 14:18] = False  # the point lens itself (A diverges)
    err = np.abs(Ab / truth - 1)[ok]
    assert err.max() < 0.01 and np.sqrt((err ** 2).mean()) < 0.003


@pytest.mark.slow
def test_binary_map_matches_quintic_blocks_outside_caustics():
    c = TINY
    cnt, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=8)
    A = cnt.astype(np.float64) * float(map_scale(c["rays"], c["window"]))
    B = 16
    nb = 512 // B
    mask = caustic_mask(c["s"], c["q"], *c["window"], margin_px=2)
    blocks_bad = mask.reshape(nb, B, nb, B).any(axis=(1, 3))
    rng = np.random.default_rng(1)
    cand = np.argwhere(~blocks_bad)
    pick = cand[rng.choice(len(cand), 24, replace=False)]
    d = 2.0 / 512
    sub = (np.arange(32) + 0.5) / 32 * B * d
    for bj, bi in pick:
        x = -1.0 + bi * B * d + sub
        y = -1.0 + bj * B * d + sub
        z = x[None, :] + 1j * y[:, None]
        truth = point_source_magnification(z, c["s"], c["q"]).mean()
        got = A[bj * B:(bj + 1) * B, bi * B:(bi + 1) * B].mean()
        assert got / truth == pytest.approx(1.0, abs=0.012)
