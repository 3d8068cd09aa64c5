"""Binary point-mass lens: geometry, lens equation, quintic images, magnification.

Test infrastructure only (see the package docstring).  All arithmetic is FP64.

Sources in the paper (McDougall & Albrow 2015):
  * sec. 4.1, parameter list: origin at the lens centre of mass, both masses on the
    first coordinate axis, separation d (called s here), mass ratio q.
  * sec. 3, Eq. 2: zeta = z - eps1/(conj(z) - conj(z1)) - eps2/(conj(z) - conj(z2)),
    eps_k the mass fractions.
  * sec. 3, text after Eq. 2: inverting Eq. 2 gives a fifth-order complex polynomial
    with 3 or 5 physical solutions.
  * sec. 3, Eqs. 3-4: image magnification 1/det J with J = d zeta / d z; total
    magnification is the sum over images (absolute values of 1/det J).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lens_setup", "lens_equation", "quintic_coefficients", "image_positions",
    "aberth_roots", "point_source_magnification", "paczynski", "disk_magnification",
]


def lens_setup(s: float, q: float):
    """Mass fractions and positions (sec. 4.1; the text's centre-of-mass origin).

    m1 = 1/(1+q) at x1 = -s q/(1+q); m2 = q/(1+q) at x2 = +s/(1+q).  The centre of
    mass m1 x1 + m2 x2 is the origin and x2 - x1 = s.
    """
    s = float(s)
    q = float(q)
    m1 = 1.0 / (1.0 + q)
    m2 = q / (1.0 + q)
    x1 = -s * q / (1.0 + q)
    x2 = s / (1.0 + q)
    return m1, m2, x1, x2


def lens_equation(z, s: float, q: float):
    """Eq. 2 for complex image positions z (FP64): returns the source position zeta."""
    m1, m2, x1, x2 = lens_setup(s, q)
    z = np.asarray(z, dtype=np.complex128)
    zc = np.conj(z)
    return z - m1 / (zc - x1) - m2 / (zc - x2)


def _pmul(a, b):
    """Product of batched polynomials with ascending coefficients on the last axis."""
    a = np.asarray(a)
    b = np.asarray(b)
    na, nb = a.shape[-1], b.shape[-1]
    shape = np.broadcast_shapes(a.shape[:-1], b.shape[:-1]) + (na + nb - 1,)
    out = np.zeros(shape, dtype=np.complex128)
    for i in range(na):
        for j in range(nb):
            out[..., i + j] += a[..., i] * b[..., j]
    return out


def _padd(a, b):
    n = max(a.shape[-1], b.shape[-1])
    shape = np.broadcast_shapes(a.shape[:-1], b.shape[:-1]) + (n,)
    out = np.zeros(shape, dtype=np.complex128)
    out[..., : a.shape[-1]] += a
    out[..., : b.shape[-1]] += b
    return out


def quintic_coefficients(zeta, s: float, q: float):
    """Fifth-degree polynomial whose roots contain the images of source zeta.

    Derived here from Eq. 2.  Conjugating Eq. 2 gives
        conj(z) = conj(zeta) + W(z),  W(z) = m1/(z-x1) + m2/(z-x2) = N(z)/D(z),
    with D = (z-x1)(z-x2) and N = (m1+m2) z - (m1 x2 + m2 x1).  Putting this back into
    Eq. 2, each deflection term becomes m_k D / P_k with P_k = (conj(zeta) - x_k) D + N,
    and clearing denominators yields
        p(z) = (zeta - z) P1 P2 + m1 D P2 + m2 D P1 = 0,   deg p = 5.
    Returns ascending coefficients, shape zeta.shape + (6,).
    """
    m1, m2, x1, x2 = lens_setup(s, q)
    zeta = np.asarray(zeta, dtype=np.complex128)
    zb = np.conj(zeta)[..., None]
    D = np.array([x1 * x2, -(x1 + x2), 1.0], dtype=np.complex128)
    N = np.array([-(m1 * x2 + m2 * x1), m1 + m2], dtype=np.complex128)
    P1 = _padd((zb - x1) * D, N[None] if zeta.ndim == 0 else np.broadcast_to(N, zb.shape[:-1] + (2,)))
    P2 = _padd((zb - x2) * D, N[None] if zeta.ndim == 0 else np.broadcast_to(N, zb.shape[:-1] + (2,)))
    lin = np.stack([zeta, -np.ones_like(zeta)], axis=-1)
    p = _pmul(lin, _pmul(P1, P2))
    p = _padd(p, m1 * _pmul(D, P2))
    p = _padd(p, m2 * _pmul(D, P1))
    if zeta.ndim == 0:
        p = p.reshape(6)
    return p


def _companion_roots(coeffs):
    """Roots of batched polynomials (ascending coefficients) via companion eigenvalues."""
    c = np.asarray(coeffs, dtype=np.complex128)
    n = c.shape[-1] - 1
    lead = c[..., -1:]
    monic = c[..., :-1] / lead
    batch = c.shape[:-1]
    comp = np.zeros(batch + (n, n), dtype=np.complex128)
    comp[..., 1:, :-1] = np.eye(n - 1)
    comp[..., :, -1] = -monic
    return np.linalg.eigvals(comp)


def _polish(coeffs, roots, iters=2):
    """Newton iterations on the polynomial (Horner evaluation of p and p')."""
    c = np.asarray(coeffs)[..., None, :]
    z = roots.copy()
    n = c.shape[-1] - 1
    for _ in range(iters):
        p = np.zeros_like(z)
        dp = np.zeros_like(z)
        for k in range(n, -1, -1):
            dp = dp * z + p
            p = p * z + c[..., k]
        ok = dp != 0
        step = np.where(ok, p / np.where(ok, dp, 1.0), 0.0)
        z = z - step
    return z


def aberth_roots(coeffs, iters=200, tol=1e-15):
    """Roots of one polynomial by the Aberth-Ehrlich simultaneous iteration.

    Independent of ``numpy.roots`` (used only to pin the companion-matrix solver).
    Starting points on a circle of radius given by the Cauchy bound, rotated off axis.
    """
    c = np.asarray(coeffs, dtype=np.complex128)
    n = len(c) - 1
    bound = 1.0 + np.max(np.abs(c[:-1] / c[-1]))
    z = 0.5 * bound * np.exp(1j * (2 * np.pi * np.arange(n) / n + 0.4))
    for _ in range(iters):
        p = np.zeros(n, dtype=np.complex128)
        dp = np.zeros(n, dtype=np.complex128)
        for k in range(n, -1, -1):
            dp = dp * z + p
            p = p * z + c[k]
        ratio = p / dp
        diff = z[:, None] - z[None, :]
        np.fill_diagonal(diff, 1.0)
        inv = 1.0 / diff
        np.fill_diagonal(inv, 0.0)
        w = ratio / (1.0 - ratio * inv.sum(axis=1))
        z = z - w
        if np.max(np.abs(w)) < tol * max(1.0, np.max(np.abs(z))):
            break
    return z


def image_positions(zeta, s: float, q: float, chunk: int = 200_000):
    """Images of point sources at zeta (any shape).

    Returns (roots[..., 5], is_image[..., 5]): all quintic roots, polished by Newton on
    the polynomial, and the mask of those that satisfy Eq. 2 itself.  The mask keeps
    the 3 or 5 roots with the smallest Eq.-2 residual (sec. 3: 3 or 5 images): 5 when
    all five residuals are below 1e-6 (1 + |zeta|), else 3 when at least three are;
    fewer only when FP64 cannot resolve an image lying on top of a lens mass.
    For q = 0 (a massless companion) the single-lens pair of images is kept.
    """
    zeta = np.asarray(zeta, dtype=np.complex128)
    flat = zeta.reshape(-1)
    roots = np.empty((flat.size, 5), dtype=np.complex128)
    for a in range(0, flat.size, chunk):
        b = min(a + chunk, flat.size)
        c = quintic_coefficients(flat[a:b], s, q)
        r = _companion_roots(c)
        roots[a:b] = _polish(c, r)
    with np.errstate(invalid="ignore", divide="ignore"):
        res = np.abs(lens_equation(roots, s, q) - flat[:, None])
    res = np.where(np.isfinite(res), res, np.inf)
    order = np.argsort(res, axis=1)
    rs = np.take_along_axis(res, order, axis=1)
    tol = 1e-6 * (1.0 + np.abs(flat))
    if float(q) == 0.0:
        # single lens: the massless companion contributes no image (two images)
        nimg = np.full(flat.size, 2)
    else:
        nvalid = np.sum(rs < tol[:, None], axis=1)
        # 5 or 3 images; fewer only when an image sits so close to a lens mass that
        # FP64 cannot resolve it (its magnification is then negligible)
        nimg = np.where(nvalid >= 5, 5, np.where(nvalid >= 3, 3, nvalid))
    rank = np.argsort(order, axis=1)
    is_image = rank < nimg[:, None]
    return roots.reshape(zeta.shape + (5,)), is_image.reshape(zeta.shape + (5,))


def point_source_magnification(zeta, s: float, q: float, return_details=False):
    """Point-source binary-lens magnification (Eqs. 3-4) at source positions zeta.

    det J = 1 - |sum_k m_k / (conj(z) - x_k)^2|^2 for each image; A = sum_j 1/|det J_j|.
    With ``return_details`` also returns the image count and the signed sum
    sum_j 1/det J_j (equal to 1 for five-image positions; used as a pin).
    """
    m1, m2, x1, x2 = lens_setup(s, q)
    roots, is_img = image_positions(zeta, s, q)
    zc = np.conj(np.where(is_img, roots, 0.5 * (x1 + x2) + 1j))
    g = m1 / (zc - x1) ** 2 + m2 / (zc - x2) ** 2
    det = 1.0 - np.abs(g) ** 2
    inv = np.where(is_img, 1.0 / det, 0.0)
    A = np.sum(np.abs(inv), axis=-1)
    if return_details:
        return A, np.sum(is_img, axis=-1), np.sum(inv, axis=-1)
    return A


def paczynski(u):
    """Single-lens point-source magnification A(u) = (u^2+2)/(u sqrt(u^2+4)) (FP64)."""
    u = np.asarray(u, dtype=np.float64)
    return (u * u + 2.0) / (u * np.sqrt(u * u + 4.0))


def disk_magnification(zeta_c, rho: float, s: float, q: float, nr: int = 16, nphi: int = 64):
    """Uniform-disk finite-source magnification (sec. 3, finite source).

    Mean of the point-source magnification over the disk |zeta - zeta_c| <= rho:
    (1/2pi) int dphi int_0^1 2x A(rho x, phi) dx, Gauss-Legendre in x = r/rho (the
    factor x absorbs the 1/r growth of A at a point lens) times a uniform periodic
    rule in angle.  Used only to synthesise light curves.
    """
    zeta_c = np.asarray(zeta_c, dtype=np.complex128)
    xg, wg = np.polynomial.legendre.leggauss(nr)
    x = 0.5 * (xg + 1.0)
    wx = 0.5 * wg * 2.0 * x
    phi = 2.0 * np.pi * (np.arange(nphi) + 0.5) / nphi
    offs = (rho * x[:, None] * np.exp(1j * phi)[None, :]).reshape(-1)
    wts = np.repeat(wx, nphi) / nphi
    pts = zeta_c.reshape(-1)[:, None] + offs[None, :]
    A = point_source_magnification(pts, s, q)
    return (A @ wts).reshape(zeta_c.shape)
