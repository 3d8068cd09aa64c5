"""Trajectory geometry and bilinear map sampling (test infrastructure only).

Sec. 4.1 parameters: u0 is the closest approach to the lens barycentre, phi (alpha
here) the trajectory angle from the positive lens axis, t0 the time of closest approach,
tE the Einstein time.  Sec. 4.2: a time t_i maps to a point on the linear trajectory,
and the magnification there is read from the map by bilinear interpolation.

Orientation (the paper does not fix it): zeta(t) = tau (cos a, sin a) + u0 (-sin a, cos a),
tau = (t - t0)/tE.  Map values sit at pixel centres, pixel i of M spanning
[c - V/2 + i V/M, c - V/2 + (i+1) V/M), so the continuous grid coordinate of a source
position is g = (zeta - c) M/V + (M/2 - 1/2) and value i sits at g = i.  Points
whose 2x2 bilinear cell is not inside the map take the single-lens
(Paczynski) magnification about the barycentre.

FP32 mirror, operation by operation.  Per trajectory, in FP64 then rounded once to binary32:
  t0' = t0 - t_ref, iE = 1/tE, ca = cos a, sa = sin a, bx = -u0 sin a, by = u0 cos a.
Per point (tt = fl32(t - t_ref), given as input), binary32 ops:
  tau = (tt - t0')*iE;  zx = tau*ca + bx;  zy = tau*sa + by;
  gx = ((zx - sx)*kx) + ox  with kx = fl32(Mx/Vx), sx = fl32(cx), ox = Mx/2 - 1/2;
  on map iff 0 <= gx < Mx-1 and 0 <= gy < My-1;  i0 = floor(gx), fx = gx - i0;
  e0 = v10 - v00, e1 = v11 - v01, ax0 = v00 + fx*e0, ax1 = v01 + fx*e1,
  A = ax0 + fy*(ax1 - ax0)       (v_ab = map[j0 + b, i0 + a]);
  off map: uu = zx*zx + zy*zy, A = (uu + 2) / sqrt(uu*(uu + 4)).
"""
from __future__ import annotations

import numpy as np

__all__ = ["traj_constants32", "map_geometry32", "sample_mirror32", "sample_exact64",
           "trajectory_positions"]

_f = np.float32


def traj_constants32(params, t_ref):
    """params [n, 4] FP64 (t0, u0, tE, alpha) -> dict of float32 arrays [n]."""
    p = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    t0, u0, tE, al = p[:, 0], p[:, 1], p[:, 2], p[:, 3]
    s, c = np.sin(al), np.cos(al)
    return dict(t0p=(t0 - t_ref).astype(_f), iE=(1.0 / tE).astype(_f), ca=c.astype(_f),
                sa=s.astype(_f), bx=(-u0 * s).astype(_f), by=(u0 * c).astype(_f))


def map_geometry32(window):
    cx, cy, vx, vy, mx, my = window
    return dict(sx=_f(cx), sy=_f(cy), kx=_f(mx / vx), ky=_f(my / vy),
                ox=_f(mx / 2 - 0.5), oy=_f(my / 2 - 0.5), mx=int(mx), my=int(my))


def sample_mirror32(amap, window, consts, tt, parts=False):
    """Binary32 samples A[n_traj, n_pts] (float32) for consts from traj_constants32.

    With ``parts`` also returns the intermediate binary32 quantities used by the
    adjoint (tau, zx, zy, onmap, fx, fy, e0, e1, ax0, ax1).
    """
    g = map_geometry32(window)
    amap = np.asarray(amap, dtype=np.float32)
    tt = np.asarray(tt, dtype=np.float32)[None, :]
    k = {n: np.asarray(v, dtype=np.float32)[:, None] for n, v in consts.items()}
    tau = (tt - k["t0p"]) * k["iE"]
    zx = tau * k["ca"] + k["bx"]
    zy = tau * k["sa"] + k["by"]
    gx = ((zx - g["sx"]) * g["kx"]) + g["ox"]
    gy = ((zy - g["sy"]) * g["ky"]) + g["oy"]
    with np.errstate(invalid="ignore"):
        on = (gx >= 0) & (gx < _f(g["mx"] - 1)) & (gy >= 0) & (gy < _f(g["my"] - 1))
    gxs = np.where(on, gx, _f(0.0))
    gys = np.where(on, gy, _f(0.0))
    fi = np.floor(gxs)
    fj = np.floor(gys)
    fx = gxs - fi
    fy = gys - fj
    i0 = fi.astype(np.int64)
    j0 = fj.astype(np.int64)
    v00 = amap[j0, i0]
    v10 = amap[j0, i0 + 1]
    v01 = amap[j0 + 1, i0]
    v11 = amap[j0 + 1, i0 + 1]
    e0 = v10 - v00
    e1 = v11 - v01
    ax0 = v00 + fx * e0
    ax1 = v01 + fx * e1
    A_on = ax0 + fy * (ax1 - ax0)
    with np.errstate(divide="ignore", invalid="ignore"):
        uu = zx * zx + zy * zy
        A_off = (uu + _f(2.0)) / np.sqrt(uu * (uu + _f(4.0)))
    A = np.where(on, A_on, A_off)
    if parts:
        return A, dict(tau=tau, zx=zx, zy=zy, onmap=on, fx=fx, fy=fy, e0=e0, e1=e1,
                       ax0=ax0, ax1=ax1, kx=g["kx"], ky=g["ky"], i0=np.where(on, i0, -1),
                       j0=np.where(on, j0, -1))
    return A


def sample_exact64(amap, window, params, t, t_ref=0.0, parts=False):
    """FP64 geometry from unrounded parameters, FP64 bilinear on the same map values.

    ``t`` are absolute FP64 times.  Same steps as the mirror, every op in FP64.
    """
    cx, cy, vx, vy, mx, my = window
    p = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    t0, u0, tE, al = (p[:, i][:, None] for i in range(4))
    amap = np.asarray(amap, dtype=np.float64)
    tau = ((np.asarray(t, dtype=np.float64) - t_ref)[None, :] - (t0 - t_ref)) / tE
    zx = tau * np.cos(al) - u0 * np.sin(al)
    zy = tau * np.sin(al) + u0 * np.cos(al)
    kx, ky = mx / vx, my / vy
    gx = (zx - cx) * kx + (mx / 2 - 0.5)
    gy = (zy - cy) * ky + (my / 2 - 0.5)
    on = (gx >= 0) & (gx < mx - 1) & (gy >= 0) & (gy < my - 1)
    gxs = np.where(on, gx, 0.0)
    gys = np.where(on, gy, 0.0)
    i0 = np.floor(gxs).astype(np.int64)
    j0 = np.floor(gys).astype(np.int64)
    fx = gxs - i0
    fy = gys - j0
    v00, v10 = amap[j0, i0], amap[j0, i0 + 1]
    v01, v11 = amap[j0 + 1, i0], amap[j0 + 1, i0 + 1]
    e0 = v10 - v00
    e1 = v11 - v01
    ax0 = v00 + fx * e0
    ax1 = v01 + fx * e1
    A_on = ax0 + fy * (ax1 - ax0)
    with np.errstate(divide="ignore", invalid="ignore"):
        uu = zx * zx + zy * zy
        A_off = (uu + 2.0) / np.sqrt(uu * (uu + 4.0))
    A = np.where(on, A_on, A_off)
    if parts:
        return A, dict(tau=tau, zx=zx, zy=zy, onmap=on, fx=fx, fy=fy, e0=e0, e1=e1,
                       ax0=ax0, ax1=ax1, kx=kx, ky=ky, i0=np.where(on, i0, -1),
                       j0=np.where(on, j0, -1))
    return A


def trajectory_positions(params, t):
    """FP64 source positions zeta(t) (complex) of one trajectory (t0, u0, tE, alpha)."""
    t0, u0, tE, al = (float(v) for v in np.asarray(params, dtype=np.float64).reshape(4))
    tau = (np.asarray(t, dtype=np.float64) - t0) / tE
    return (tau * np.cos(al) - u0 * np.sin(al)) + 1j * (tau * np.sin(al) + u0 * np.cos(al))
