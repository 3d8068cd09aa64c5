"""Pins of oracle.profiles: limb-darkened source-profile weights (sec. 4.1 finite-source
maps with fixed limb darkening) and the radius stack."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.maps import disk_pixel_weights, map_scale, normalize_convolve_exact64
from oracle.profiles import ld_intensity, ld_pixel_weights, ld_rect_integral, stack_rhos
from oracle.rays import rayshoot_mirror32_c

D2048 = 3 / 2048


@pytest.mark.parametrize("rho,dx,dy", [(2e-3, D2048, D2048), (0.01, 3 / 1024, 3 / 1024),
                                       (0.004, 0.003, 0.002), (0.05, D2048, D2048)])
def test_zero_gamma_is_the_uniform_disk(rho, dx, dy):
    # analytic circle-rectangle areas vs this module's quadrature
    u = disk_pixel_weights(rho, dx, dy)
    w = ld_pixel_weights(rho, dx, dy, 0.0)
    assert w.shape == u.shape
    assert np.abs(w - u).max() < 1e-13


@pytest.mark.parametrize("gamma", [0.0, 0.353, 0.53, 1.0])
@pytest.mark.parametrize("rho,d", [(2e-3, D2048), (0.0316, D2048), (0.3, 3 / 256)])
def test_profile_integrates_to_disk_area(rho, d, gamma):
    # the linear law has unit mean brightness over the disk, so the raw integrals over
    # pi rho^2 sum to 1 without renormalisation
    w = ld_pixel_weights(rho, d, d, gamma, normalise=False)
    assert w.sum() == pytest.approx(1.0, abs=1e-12)


def test_intensity_law_values():
    rho = 0.2
    assert ld_intensity(0.0, rho, 0.53) == pytest.approx(1 + 0.53 / 2, abs=1e-15)
    assert ld_intensity(rho, rho, 0.53) == pytest.approx(1 - 0.53, abs=1e-15)
    assert ld_intensity(1.01 * rho, rho, 0.53) == 0.0
    # unit mean over the disk, by radial quadrature
    m, _ = integrate.quad(lambda r: ld_intensity(r, rho, 0.53) * 2 * math.pi * r, 0, rho)
    assert m / (math.pi * rho * rho) == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("rect", [(0.0, 0.3, 0.1, 0.5), (-0.2, 0.2, -0.2, 0.2), (0.5, 0.9, -0.3, 0.1),
                                  (0.7, 1.2, 0.0, 0.4)])
def test_rect_integral_matches_dblquad(rect):
    rho, gamma = 1.0, 0.53
    x1, x2, y1, y2 = rect

    def f(y, x):
        return float(ld_intensity(math.hypot(x, y), rho, gamma))

    def ylo(x):
        return max(y1, -math.sqrt(max(rho * rho - x * x, 0.0)))

    def yhi(x):
        return max(ylo(x), min(y2, math.sqrt(max(rho * rho - x * x, 0.0))))

    ref, err = integrate.dblquad(f, max(x1, -rho), min(x2, rho), ylo, yhi, epsabs=1e-13, epsrel=1e-12)
    assert ld_rect_integral(x1, x2, y1, y2, rho, gamma) == pytest.approx(ref, abs=1e-11)


@pytest.mark.parametrize("rho,dx,dy", [(2e-3, D2048, D2048), (0.01, 3 / 1024, 3 / 1024),
                                       (0.004, 0.003, 0.002)])
def test_weights_match_supersampling(rho, dx, dy):
    gamma = 0.53
    w = ld_pixel_weights(rho, dx, dy, gamma)
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    Ry, Rx = (w.shape[0] - 1) // 2, (w.shape[1] - 1) // 2
    n = 1500
    xs = (np.arange(-(2 * Rx + 1) * n // 2, (2 * Rx + 1) * n // 2) + 0.5) * dx / n
    ys = (np.arange(-(2 * Ry + 1) * n // 2, (2 * Ry + 1) * n // 2) + 0.5) * dy / n
    X, Y = np.meshgrid(xs, ys)
    I = ld_intensity(np.hypot(X, Y), rho, gamma)
    ii = np.floor(X / dx + 0.5).astype(int) + Rx
    jj = np.floor(Y / dy + 0.5).astype(int) + Ry
    ws = np.zeros_like(w)
    np.add.at(ws, (jj, ii), I)
    ws /= ws.sum()
    assert np.abs(ws - w).max() < 3e-5
    assert np.array_equal(w, w[::-1, :]) and np.array_equal(w, w[:, ::-1])
    if dx == dy:
        assert np.abs(w - w.T).max() < 1e-15


def test_limb_darkening_moves_weight_to_the_centre():
    rho, d = 0.05, D2048
    u = ld_pixel_weights(rho, d, d, 0.0)
    w = ld_pixel_weights(rho, d, d, 0.53)
    c = (u.shape[0] // 2, u.shape[1] // 2)
    assert w[c] > u[c] * 1.2  # centre brightness 1 + Gamma/2 over the mean
    assert w[c[0], 0] < u[c[0], 0]  # limb pixel dimmer


def test_stack_radii():
    r = stack_rhos()
    assert len(r) == 7
    assert r[0] == pytest.approx(1e-3, rel=1e-15) and r[-1] == pytest.approx(1.0, rel=1e-15)
    assert np.allclose(np.diff(np.log10(r)), 0.5, atol=1e-14)


@pytest.mark.parametrize("rho", [0.1, 0.3])
def test_single_lens_centred_limb_darkened_source(rho):
    # q = 0, source centred on the lens: a uniform disk of radius r maps to an image
    # annulus of area pi r sqrt(r^2+4), so the profile-weighted magnification is
    # (1/rho^2) int_0^rho I(r) d/dr[r sqrt(r^2+4)] dr.  The window is shifted by half a
    # pixel so that a pixel centre sits on the lens.
    gamma = 0.53
    nx = 256
    d = 2.0 / nx
    window = (d / 2, d / 2, 2.0, 2.0, nx, nx)
    rays = (0.0, 0.0, 4.0, 4.0, 4000, 4000)
    counts, _ = rayshoot_mirror32_c(1.0, 0.0, rays, window, nthreads=8)
    w = ld_pixel_weights(rho, d, d, gamma)
    A = normalize_convolve_exact64(counts, map_scale(rays, window, fp32=False), w)
    ref, _ = integrate.quad(lambda r: ld_intensity(r, rho, gamma) * (2 * r * r + 4) / math.sqrt(r * r + 4),
                            0, rho, epsabs=1e-13)
    ref /= rho * rho
    assert A[nx // 2 - 1, nx // 2 - 1] == pytest.approx(ref, rel=3e-3)
    # and it differs from the uniform disk's sqrt(rho^2+4)/rho by more than that
    assert abs(ref / (math.sqrt(rho * rho + 4) / rho) - 1) > 1e-2
