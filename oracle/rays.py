"""Inverse ray shooting into a source-plane count histogram (test infrastructure only).

The map-building method is ray shooting (the family of magnification-map methods the
paper cites in sec. 3: Kayser 1986, Bennett 1996, Dong 2006): shoot a regular lattice
of image-plane rays through the binary-lens equation (Eq. 2, lens placement of
sec. 4.1) and count, for each source-plane pixel, the rays that land in it.  The
count times the no-lens ray density gives the magnification (done in ``maps``).

Grids are tuples (cx, cy, wx, wy, nx, ny): centre, full widths, counts (even).

Three implementations:
  * ``rayshoot_mirror32_numpy``: FP32 mirror in numpy float32 (each ufunc op is one
    correctly rounded binary32 op, no fused multiply-add).
  * ``rayshoot_mirror32_c``: the same steps in plain C (``rays_mirror32.c``), written
    separately; the two must agree bit for bit (pin).
  * ``rayshoot_exact64``: the same formulas in FP64 from unrounded constants.

FP32 mirror, step by step:
  lens constants m1, m2, x1, x2 from ``lens.lens_setup`` in FP64, rounded once;
  lattice spacing h = fl32(W/N), pixel scale k = fl32(M/V), centres fl32(c);
  ray i: g = (i - N/2) + 0.5 (exact), x = cx + g*h (two rounded ops);
  1/(conj z - x_k) = (z - x_k)/|z - x_k|^2 for real x_k, so with d_k = x - x_k,
  r_k = d_k*d_k + y*y and a_k = m_k/r_k:  zx = (x - a1*d1) - a2*d2,
  zy = (y - a1*y) - a2*y;  v = (zeta - s)*k;  bin by the symmetric rule
  v >= 0 -> M/2 + floor(v) when v < M/2;  v < 0 -> M/2 - 1 - floor(-v) when -v < M/2.
The symmetric rule gives bin(-v) = M - 1 - bin(v) for every v != 0, which makes the
histogram exactly mirror-symmetric about the lens axis (pin) apart from rays with
v_y == 0, which are counted separately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .lens import lens_setup

__all__ = ["f32_constants", "ray_positions_mirror32", "rayshoot_mirror32_numpy", "rayshoot_mirror32_c",
           "rayshoot_exact64", "ray_stats_template"]

_f = np.float32


def f32_constants(s, q, rays, window):
    """FP64 constants rounded once to binary32 (dict of np.float32)."""
    m1, m2, x1, x2 = lens_setup(s, q)
    cx, cy, wx, wy, nx, ny = rays
    sx, sy, vx, vy, mx, my = window
    return dict(m1=_f(m1), m2=_f(m2), x1=_f(x1), x2=_f(x2), cx=_f(cx), cy=_f(cy),
                hx=_f(wx / nx), hy=_f(wy / ny), sx=_f(sx), sy=_f(sy),
                kx=_f(mx / vx), ky=_f(my / vy))


def ray_stats_template():
    return dict(out=0, nonfinite=0, zero_axis=0)


def _bin_f32(v, m):
    """Symmetric bin rule on float32 v; returns (index int64, inside bool)."""
    half = _f(m // 2)
    pos = v >= _f(0.0)
    with np.errstate(invalid="ignore"):
        fpos = np.floor(np.where(pos, v, _f(0.0)))
        fneg = np.floor(np.where(pos, _f(0.0), -v))
    inside = np.where(pos, v < half, -v < half)
    idx = np.where(pos, m // 2 + fpos.astype(np.int64), m // 2 - 1 - fneg.astype(np.int64))
    return idx, inside


def ray_positions_mirror32(s, q, rays, window, rows):
    """Binary32 source positions and scaled window offsets of lattice rows j0..j1-1.

    Returns (zx, zy, vx, vy), each float32 [rows, nx].
    """
    c = f32_constants(s, q, rays, window)
    nx, ny = int(rays[4]), int(rays[5])
    a, b = rows
    gx = (np.arange(nx, dtype=np.int64) - nx // 2).astype(np.float32) + _f(0.5)
    x = (c["cx"] + gx * c["hx"])[None, :]
    gy = (np.arange(a, b, dtype=np.int64) - ny // 2).astype(np.float32) + _f(0.5)
    y = (c["cy"] + gy * c["hy"])[:, None]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        d1 = x - c["x1"]
        d2 = x - c["x2"]
        yy = y * y
        r1 = d1 * d1 + yy
        r2 = d2 * d2 + yy
        a1 = c["m1"] / r1
        a2 = c["m2"] / r2
        zx = (x - a1 * d1) - a2 * d2
        zy = (y - a1 * y) - a2 * y
        vx = (zx - c["sx"]) * c["kx"]
        vy = (zy - c["sy"]) * c["ky"]
    return zx, zy, vx, vy


def rayshoot_mirror32_numpy(s, q, rays, window, rows=None, chunk_rows=64):
    """FP32 mirror in numpy.  ``rows`` = (j0, j1) restricts to lattice rows j0..j1-1."""
    ny = int(rays[5])
    mx, my = int(window[4]), int(window[5])
    j0, j1 = rows if rows is not None else (0, ny)
    counts = np.zeros(my * mx, dtype=np.uint64)
    st = ray_stats_template()
    for a in range(j0, j1, chunk_rows):
        b = min(a + chunk_rows, j1)
        _, _, vx, vy = ray_positions_mirror32(s, q, rays, window, (a, b))
        fin = np.isfinite(vx) & np.isfinite(vy)
        ix, inx = _bin_f32(vx, mx)
        iy, iny = _bin_f32(vy, my)
        inside = fin & inx & iny
        st["nonfinite"] += int(np.count_nonzero(~fin))
        st["out"] += int(np.count_nonzero(fin & ~(inx & iny)))
        st["zero_axis"] += int(np.count_nonzero(inside & (vy == 0)))
        flat = iy[inside] * mx + ix[inside]
        counts += np.bincount(flat, minlength=my * mx).astype(np.uint64)
    return counts.reshape(my, mx).astype(np.uint32), st


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in
                ("m1", "m2", "x1", "x2", "cx", "cy", "hx", "hy", "sx", "sy", "kx", "ky")] + \
               [(n, ctypes.c_int32) for n in ("nx", "ny", "mx", "my")]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from . import build as _build
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_rayshoot_mirror32.restype = ctypes.c_int
        lib.oracle_rayshoot_mirror32.argtypes = [
            ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        _LIB = lib
    return _LIB


def rayshoot_mirror32_c(s, q, rays, window, rows=None, nthreads=1, counts=None):
    """FP32 mirror in C (``rays_mirror32.c``).  Accumulates into ``counts`` if given."""
    c = f32_constants(s, q, rays, window)
    p = _Params(*(float(c[k]) for k in ("m1", "m2", "x1", "x2", "cx", "cy", "hx", "hy",
                                         "sx", "sy", "kx", "ky")),
                int(rays[4]), int(rays[5]), int(window[4]), int(window[5]))
    mx, my = int(window[4]), int(window[5])
    if counts is None:
        counts = np.zeros((my, mx), dtype=np.uint32)
    stats = np.zeros(3, dtype=np.uint64)
    j0, j1 = rows if rows is not None else (0, int(rays[5]))
    rc = _lib().oracle_rayshoot_mirror32(ctypes.byref(p), counts.ctypes.data, stats.ctypes.data,
                                         j0, j1, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_rayshoot_mirror32 failed: {rc}")
    return counts, dict(out=int(stats[0]), nonfinite=int(stats[1]), zero_axis=int(stats[2]))


def rayshoot_exact64(s, q, rays, window, rows=None, chunk_rows=64):
    """The same steps in FP64 from unrounded constants (h = W/N, k = M/V)."""
    m1, m2, x1, x2 = lens_setup(s, q)
    cx, cy, wx, wy, nx, ny = rays
    sx, sy, vxw, vyw, mx, my = window
    nx, ny, mx, my = int(nx), int(ny), int(mx), int(my)
    hx, hy = wx / nx, wy / ny
    kx, ky = mx / vxw, my / vyw
    j0, j1 = rows if rows is not None else (0, ny)
    counts = np.zeros(my * mx, dtype=np.uint64)
    st = ray_stats_template()
    x = cx + ((np.arange(nx) - nx // 2) + 0.5) * hx
    d1 = x - x1
    d2 = x - x2
    for a in range(j0, j1, chunk_rows):
        b = min(a + chunk_rows, j1)
        y = (cy + ((np.arange(a, b) - ny // 2) + 0.5) * hy)[:, None]
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            r1 = d1[None, :] ** 2 + y * y
            r2 = d2[None, :] ** 2 + y * y
            zx = x[None, :] - m1 * d1[None, :] / r1 - m2 * d2[None, :] / r2
            zy = y - m1 * y / r1 - m2 * y / r2
            vx = (zx - sx) * kx
            vy = (zy - sy) * ky
        fin = np.isfinite(vx) & np.isfinite(vy)
        pos_x = vx >= 0
        pos_y = vy >= 0
        with np.errstate(invalid="ignore"):
            ix = np.where(pos_x, mx // 2 + np.floor(np.where(fin, vx, 0)),
                          mx // 2 - 1 - np.floor(np.where(fin, -vx, 0)))
            iy = np.where(pos_y, my // 2 + np.floor(np.where(fin, vy, 0)),
                          my // 2 - 1 - np.floor(np.where(fin, -vy, 0)))
        inside = fin & (np.abs(vx) < mx // 2) & (np.abs(vy) < my // 2)
        st["nonfinite"] += int(np.count_nonzero(~fin))
        st["out"] += int(np.count_nonzero(fin & ~inside))
        st["zero_axis"] += int(np.count_nonzero(inside & (vy == 0)))
        flat = iy[inside].astype(np.int64) * mx + ix[inside].astype(np.int64)
        counts += np.bincount(flat, minlength=my * mx).astype(np.uint64)
    return counts.reshape(my, mx), st
