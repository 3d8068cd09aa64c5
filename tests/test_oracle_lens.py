"""Pins of oracle.lens: quintic images and point-source magnification (Eqs. 2-4)."""
import numpy as np
import pytest

from oracle.lens import (aberth_roots, disk_magnification, image_positions, lens_equation,
                         lens_setup, paczynski, point_source_magnification,
                         quintic_coefficients)


def test_lens_setup_centre_of_mass_and_separation():
    for s, q in [(1.0, 1e-3), (0.8, 5e-3), (2.5, 1.0), (0.3, 0.1)]:
        m1, m2, x1, x2 = lens_setup(s, q)
        assert m1 + m2 == pytest.approx(1.0, abs=1e-15)
        assert m1 * x1 + m2 * x2 == pytest.approx(0.0, abs=1e-15)
        assert x2 - x1 == pytest.approx(s, rel=1e-15)
        assert m2 / m1 == pytest.approx(q, rel=1e-14)


def test_companion_roots_match_aberth():
    rng = np.random.default_rng(3)
    for _ in range(20):
        s = 10 ** rng.uniform(-0.5, 0.5)
        q = 10 ** rng.uniform(-4, 0)
        zeta = complex(*rng.uniform(-1, 1, 2))
        c = quintic_coefficients(zeta, s, q)
        r1 = np.sort_complex(np.roots(c[::-1]))
        r2 = aberth_roots(c)
        # match each numpy root with the nearest Aberth root
        d = np.abs(r1[:, None] - r2[None, :]).min(axis=1)
        assert d.max() < 1e-9 * max(1.0, np.abs(r1).max())


def test_images_satisfy_lens_equation_and_count():
    rng = np.random.default_rng(5)
    for s, q in [(1.0, 1e-3), (0.7, 0.5), (1.3, 0.1)]:
        zeta = rng.uniform(-1, 1, 3000) + 1j * rng.uniform(-1, 1, 3000)
        roots, img = image_positions(zeta, s, q)
        n = img.sum(axis=1)
        assert set(np.unique(n)) <= {3, 5}
        res = np.abs(lens_equation(roots, s, q) - zeta[:, None])
        # images close to a lens mass are ill-conditioned in Eq. 2 (|dzeta/dz| large)
        assert res[img].max() < 1e-7


def test_five_image_signed_magnification_is_one():
    # sum_j 1/det J_j = 1 for five-image positions (Witt & Mao 1995 invariant)
    rng = np.random.default_rng(7)
    s, q = 1.0, 0.3
    zeta = rng.uniform(-0.4, 0.4, 4000) + 1j * rng.uniform(-0.4, 0.4, 4000)
    _, n, signed = point_source_magnification(zeta, s, q, return_details=True)
    assert (n == 5).sum() > 100
    assert np.abs(signed[n == 5] - 1.0).max() < 1e-8


def test_single_lens_limits():
    rng = np.random.default_rng(9)
    zeta = rng.uniform(-1, 1, 2000) + 1j * rng.uniform(-1, 1, 2000)
    u = np.abs(zeta)
    A = point_source_magnification(zeta, 1.0, 0.0)
    assert np.abs(A / paczynski(u) - 1).max() < 1e-9
    # q -> 0 with a far companion: Paczynski about the primary away from the
    # companion's caustic (near x2 - 1/x2)
    s, q = 3.0, 1e-8
    m1, m2, x1, x2 = lens_setup(s, q)
    A = point_source_magnification(zeta, s, q)
    far = np.abs(zeta - (x2 - 1 / x2)) > 0.2
    assert np.abs(A[far] / paczynski(np.abs(zeta[far] - x1)) - 1).max() < 1e-5


def test_magnification_mirror_symmetry():
    rng = np.random.default_rng(11)
    zeta = rng.uniform(-1, 1, 1000) + 1j * rng.uniform(0.05, 1, 1000)
    A1 = point_source_magnification(zeta, 0.9, 0.02)
    A2 = point_source_magnification(np.conj(zeta), 0.9, 0.02)
    assert np.abs(A1 / A2 - 1).max() < 1e-9


def test_disk_magnification_centred_on_single_lens():
    # a uniform disk of radius rho centred on a point lens: the images of the disk
    # fill the annulus r+- = (+-rho + sqrt(rho^2+4))/2, so A = sqrt(rho^2+4)/rho
    for rho in (0.01, 0.1, 0.5):
        A = disk_magnification(np.array([0j]), rho, 1.0, 0.0, nr=32, nphi=8)
        assert A[0] == pytest.approx(np.sqrt(rho * rho + 4) / rho, rel=1e-3)
