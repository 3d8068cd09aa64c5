"""Critical curves, caustics and the caustic-pixel mask (FP64).

Test infrastructure only.  The paper's map comparisons and the map tolerance are
stated outside caustic pixels; the paper never defines the term, so this module fixes
the reading used here: a pixel is a caustic pixel when it lies within
``margin`` pixels (Chebyshev distance, in pixel-centre units) of a point of the
point-source caustic, plus the finite-source radius in pixels for convolved maps.

Critical curves follow from Eq. 4: det J = 0 means |sum_k m_k/(conj z - x_k)^2| = 1, i.e.
sum_k m_k/(z - x_k)^2 = exp(-i phi) for some phase phi.  Clearing denominators,
    m1 (z - x2)^2 + m2 (z - x1)^2 - exp(-i phi) (z - x1)^2 (z - x2)^2 = 0,
a quartic for each phi; its roots trace the critical curves and Eq. 2 maps them to the
caustics.
"""
from __future__ import annotations

import numpy as np

from .lens import lens_setup, lens_equation, _companion_roots, _pmul, _padd

__all__ = ["critical_curve_points", "caustic_points", "caustic_mask", "image_count_mask"]

def critical_curve_points(s: float, q: float, nphi: int):
    """Critical-curve points for nphi equally spaced phases; returns [nphi, 4] complex."""
    m1, m2, x1, x2 = lens_setup(s, q)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    e = np.exp(-1j * phi)[:, None]
    A1 = np.array([x1 * x1, -2 * x1, 1.0], dtype=np.complex128)  # (z-x1)^2
    A2 = np.array([x2 * x2, -2 * x2, 1.0], dtype=np.complex128)  # (z-x2)^2
    base = _padd(m1 * A2, m2 * A1)[None, :]
    prod = _pmul(A1, A2)[None, :]
    coeffs = _padd(np.broadcast_to(base, (nphi, 3)), -e * prod)
    return _companion_roots(coeffs)


def caustic_points(s: float, q: float, nphi: int):
    """Caustic points (Eq. 2 applied to critical-curve points), [nphi, 4] complex."""
    return lens_equation(critical_curve_points(s, q, nphi), s, q)


def caustic_mask(s: float, q: float, cx: float, cy: float, wx: float, wy: float,
                 nx: int, ny: int, margin_px: int = 2, rho: float = 0.0,
                 max_step_px: float = 0.25, nphi0: int = 4096, nphi_max: int = 1 << 21):
    """Boolean [ny, nx] mask of caustic pixels of a map window.

    Pixel (j, i) has centre (cx - wx/2 + (i + 0.5) dx, cy - wy/2 + (j + 0.5) dy).  The
    caustic is sampled until every sample has a sample of the next phase within
    ``max_step_px`` pixels; every pixel within margin_px + ceil(rho/d) of a sample
    (Chebyshev distance) is marked.
    """
    dx = wx / nx
    dy = wy / ny
    nphi = nphi0
    while True:
        c = caustic_points(s, q, nphi)
        nxt = np.concatenate([c[1:], c[:1]], axis=0)
        # distance from each sample to the nearest sample of the next phase
        step = np.min(np.abs(nxt[:, None, :] - c[:, :, None]), axis=2)
        steppx = np.max(step) / min(dx, dy)
        if steppx <= max_step_px or nphi >= nphi_max:
            break
        nphi *= 2
    gx = (c.real.ravel() - (cx - wx / 2)) / dx - 0.5
    gy = (c.imag.ravel() - (cy - wy / 2)) / dy - 0.5
    mx = margin_px + int(np.ceil(rho / dx))
    my = margin_px + int(np.ceil(rho / dy))
    mask = np.zeros((ny, nx), dtype=bool)
    ic = np.rint(gx).astype(np.int64)
    jc = np.rint(gy).astype(np.int64)
    keep = (ic >= -mx - 1) & (ic <= nx + mx) & (jc >= -my - 1) & (jc <= ny + my)
    ic, jc = ic[keep], jc[keep]
    for dj in range(-my - 1, my + 2):
        for di in range(-mx - 1, mx + 2):
            ii = ic + di
            jj = jc + dj
            ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
            mask[jj[ok], ii[ok]] = True
    return mask


def image_count_mask(s: float, q: float, cx: float, cy: float, wx: float, wy: float,
                     nx: int, ny: int, sub: int = 4):
    """Pixels where the number of images differs among sub x sub interior samples.

    A caustic separates regions of 3 and 5 images, so such pixels are crossed by it.
    Used to pin ``caustic_mask`` (it must cover all of them).  Cost nx*ny*sub^2 quintics.
    """
    from .lens import point_source_magnification
    dx = wx / nx
    dy = wy / ny
    off = (np.arange(sub) + 0.5) / sub
    xs = cx - wx / 2 + (np.arange(nx)[:, None] + off[None, :]) * dx  # [nx, sub]
    ys = cy - wy / 2 + (np.arange(ny)[:, None] + off[None, :]) * dy  # [ny, sub]
    z = xs[None, :, None, :] + 1j * ys[:, None, :, None]  # [ny, nx, sub, sub]
    _, n, _ = point_source_magnification(z, s, q, return_details=True)
    n = n.reshape(ny, nx, sub * sub)
    return n.min(axis=2) != n.max(axis=2)
