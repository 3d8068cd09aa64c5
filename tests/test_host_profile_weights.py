"""Host logic of the library without a device: the limb-darkened pixel weights it
convolves with (closed-form hemisphere volumes over each pixel) against the oracle's
quadrature of the same integrals."""
import numpy as np
import pytest

import paper_1511_01157_amd as M
from oracle.maps import disk_pixel_weights
from oracle.profiles import ld_pixel_weights, stack_rhos

D2048 = 3 / 2048


@pytest.mark.parametrize("gamma", [0.0, 0.353, 0.53, 1.0])
@pytest.mark.parametrize("rho,dx,dy", [(2e-3, D2048, D2048), (0.0316, D2048, D2048),
                                       (0.004, 0.003, 0.002), (0.1, D2048, D2048),
                                       (0.3, 3 / 256, 3 / 256)])
def test_library_weights_match_oracle_quadrature(rho, dx, dy, gamma):
    w = M.profile_weights(rho, dx, dy, gamma)
    o = ld_pixel_weights(rho, dx, dy, gamma)
    assert w.shape == o.shape
    assert abs(w.sum() - 1.0) < 1e-12
    assert np.abs(w - o).max() < 1e-12 * max(1.0, 1.0 / o.max()) * o.max()


def test_library_uniform_weights_match_analytic_areas():
    for rho in (2e-3, 0.01, 0.05):
        w = M.profile_weights(rho, D2048, D2048, 0.0)
        u = disk_pixel_weights(rho, D2048, D2048)
        assert w.shape == u.shape and np.abs(w - u).max() < 1e-13


def test_identity_and_small_radius():
    assert np.array_equal(M.profile_weights(0.0, D2048, D2048, 0.53), np.ones((1, 1)))
    w = M.profile_weights(1e-3, 3 / 1024, 3 / 1024, 0.53)  # disk inside its own pixel
    assert np.array_equal(w, np.ones((1, 1)))


def test_stack_radii_stencils():
    # the seven stack radii at a 2048^2 map over 3 units: stencil half-widths R = ceil(rho/d + 1/2)
    # (outer rings that the disk misses trimmed)
    rs = [M.profile_weights(r, D2048, D2048, 0.53).shape[0] // 2 for r in stack_rhos()[:5]]
    assert rs == [1, 2, 7, 22, 68]
