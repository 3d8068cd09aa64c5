"""Shared helpers of the GPU parity tests: oracle-built inputs and comparisons.

Every input handed to both the HIP path and the oracle comes from the seeded
generators or from the oracle itself, never from the HIP path.
"""
from __future__ import annotations

import sys

import numpy as np

import workloads as W
from oracle.maps import disk_pixel_weights, map_scale, normalize_convolve_mirror32
from oracle.rays import rayshoot_mirror32_c


def note(msg):
    """Name the case before a GPU step (flushed, so it survives a lost box)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def oracle_map(s, q, rays, window, rho, nthreads=16):
    counts, st = rayshoot_mirror32_c(s, q, rays, window, nthreads=nthreads)
    dx, dy = window[2] / window[4], window[3] / window[5]
    amap = normalize_convolve_mirror32(counts, map_scale(rays, window), disk_pixel_weights(rho, dx, dy))
    return counts, st, amap


def events(name, idx):
    return [W.load_lightcurve(name, e) for e in idx]


def rel_err(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)
