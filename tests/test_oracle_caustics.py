"""Pins of oracle.caustics: critical curves (det J = 0) and the caustic mask."""
import numpy as np

from oracle.caustics import caustic_mask, critical_curve_points, image_count_mask
from oracle.lens import lens_setup


def test_critical_points_have_zero_jacobian():
    for s, q in [(1.0, 1e-3), (0.8, 5e-3), (2.0, 0.5)]:
        m1, m2, x1, x2 = lens_setup(s, q)
        z = critical_curve_points(s, q, 512).ravel()
        g = m1 / (np.conj(z) - x1) ** 2 + m2 / (np.conj(z) - x2) ** 2
        assert np.abs(1 - np.abs(g) ** 2).max() < 1e-9


def test_single_lens_critical_curve_is_einstein_ring():
    z = critical_curve_points(1.0, 1e-12, 256).ravel()
    m1, m2, x1, x2 = lens_setup(1.0, 1e-12)
    r = np.abs(z - x1)
    assert np.sort(r)[len(r) // 2:].min() > 0.999  # half the roots sit on the ring


def test_caustic_mask_covers_image_count_changes():
    for s, q in [(1.0, 1e-3), (0.8, 0.05)]:
        args = (0.0, 0.0, 0.6, 0.6, 96, 96)
        ic = image_count_mask(s, q, *args, sub=4)
        cm = caustic_mask(s, q, *args, margin_px=1)
        assert ic.sum() > 0
        assert not (ic & ~cm).any()
