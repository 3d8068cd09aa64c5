"""Pins of oracle.fsmag, the image-centred finite-source magnification (sec. 5), against
results it shares no code with: the single-lens disk integral reduced to one dimension
(the radial integral of A(u) u is u sqrt(u^2 + 4)/2 in closed form; Gauss-Legendre over
the angle), the point-source magnification of the quintic (the far branch), the
quintic disk average away from the caustic, and plain uniform ray shooting over the
whole image plane across caustics.  Tolerances: the method's own error at its default
512 x 512 cells per region (about 1e-4; a few 1e-4 with the lens on the source limb)
and the statistical error of the brute-force reference."""
import math

import numpy as np
import pytest

from oracle.caustics import caustic_points
from oracle.fsmag import FsOptions, brute_force_fs, fs_magnification, single_lens_disk
from oracle.lens import disk_magnification, point_source_magnification

SINGLE = (3.0, 1e-10)  # a point lens: a 1e-10 companion far off (its caustic near 2.67)


@pytest.mark.parametrize("gamma", [0.0, 0.53])
@pytest.mark.parametrize("b", [0.0, 0.05, 0.2, 0.5])
def test_single_lens_against_the_disk_integral(gamma, b):
    A = fs_magnification(b, 0.1, gamma, *SINGLE)
    ref = single_lens_disk(b, 0.1, gamma)
    assert abs(A / ref - 1) < 2e-4, (A, ref)


def test_single_lens_with_the_lens_on_the_limb():
    for gamma in (0.0, 0.53):
        A = fs_magnification(0.1, 0.1, gamma, *SINGLE)
        assert abs(A / single_lens_disk(0.1, 0.1, gamma) - 1) < 5e-4


def test_uniform_disk_centred_on_the_lens_closed_form():
    rho = 0.07
    A = fs_magnification(0.0, rho, 0.0, *SINGLE)
    assert abs(A / (math.sqrt(rho * rho + 4) / rho) - 1) < 1e-5


def test_far_sources_take_the_point_source_magnification():
    s, q = 0.8, 5e-3
    for z in (0.6 + 0.5j, -0.9 - 0.2j):
        A, d = fs_magnification(z, 0.01, 0.53, s, q, details=True)
        assert d["point_source"]
        assert A == float(point_source_magnification(np.array([z]), s, q)[0])


def _cusp(s, q):
    cc = np.asarray(caustic_points(s, q, 4096)).reshape(-1)
    cc = cc[np.isfinite(cc)]
    return cc[np.argmax(cc.real)], cc


@pytest.mark.parametrize("s,q", [(1.0, 1e-2), (0.8, 5e-3), (1.2, 0.3)])
def test_near_the_caustic_against_the_disk_average(s, q):
    """A few radii from the caustic the point-source magnification is smooth over the
    disk, so the quintic disk average (Gauss-Legendre x angles) is accurate."""
    c0, cc = _cusp(s, q)
    rho = 0.02
    z = c0 + 6 * rho * 1j
    assert np.min(np.abs(cc - z)) < 10 * rho                 # the image-centred branch
    A = fs_magnification(z, rho, 0.0, s, q)
    ref = complex(disk_magnification(np.array([z]), rho, s, q, nr=48, nphi=256)[0]).real
    assert abs(A / ref - 1) < 5e-4, (A, ref)


@pytest.mark.parametrize("s,q", [(0.8, 5e-3), (1.2, 0.3)])
def test_across_the_caustic_against_brute_force(s, q):
    """A source straddling the caustic at a cusp (images merging at the critical curve)
    against uniform ray shooting over the image plane (3000^2 rays over [-2.2, 2.2]^2,
    statistical error about 1.5e-3 at rho = 0.05)."""
    c0, _ = _cusp(s, q)
    rho = 0.05
    z = c0 + 0.5 * rho * 1j
    for gamma in (0.0, 0.53):
        A = fs_magnification(z, rho, gamma, s, q)
        ref = brute_force_fs(z, rho, gamma, s, q, (0.0, 0.0, 2.2), 3000)
        assert abs(A / ref - 1) < 4e-3, (gamma, A, ref)


def test_grazing_source_finds_the_small_images():
    """A source just inside the caustic near a fold: the two extra images are seeded
    from the critical points, so the magnification jumps above the outside value."""
    s, q = 1.2, 0.3
    c0, cc = _cusp(s, q)
    rho = 0.02
    out = fs_magnification(c0 + 1.05 * rho, rho, 0.0, s, q)   # just outside the cusp
    inn = fs_magnification(c0 - 0.9 * rho, rho, 0.0, s, q)    # the disk straddles it
    assert inn > out
    ref = brute_force_fs(c0 - 0.9 * rho, rho, 0.0, s, q, (0.0, 0.0, 2.2), 3000)
    assert abs(inn / ref - 1) < 5e-3
