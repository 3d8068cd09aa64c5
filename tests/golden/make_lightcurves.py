"""Write the true magnifications of the synthetic light curves (calls only the oracle).

For every event of the tiny / large / sqgrid / batched workloads: source positions
along the truth trajectory (sec. 4.1 parameters), then the point-source
binary-lens magnification from the quintic images (Eqs. 2-4).  For a finite source
(rho > 0) points within 10 rho of the caustic (the proximity rule the paper uses for
its finite-source refinement, sec. 5) take the uniform-disk average .
Output: tests/golden/lc_amag_<name>.npz with one array e<event> per event.

Run:  python tests/golden/make_lightcurves.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
from scipy.spatial import cKDTree

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.lens import point_source_magnification, disk_magnification  # noqa: E402
from oracle.caustics import caustic_points  # noqa: E402
from oracle.sampling import trajectory_positions  # noqa: E402


def event_magnification(tr, t):
    p = np.array([tr["t0"], tr["u0"], tr["tE"], tr["alpha"]])
    zeta = trajectory_positions(p, t)
    A = point_source_magnification(zeta, tr["s"], tr["q"])
    rho = tr["rho"]
    nfs = 0
    if rho > 0:
        c = caustic_points(tr["s"], tr["q"], 8192).ravel()
        tree = cKDTree(np.stack([c.real, c.imag], axis=1))
        dist, _ = tree.query(np.stack([zeta.real, zeta.imag], axis=1))
        near = dist < 10.0 * rho
        nfs = int(near.sum())
        if nfs:
            A[near] = disk_magnification(zeta[near], rho, tr["s"], tr["q"], nr=8, nphi=32)
    return A, nfs


def main(names):
    for name in names:
        t0 = time.time()
        trs = W.truths(name)
        out = {}
        nfs_tot = 0
        for e, tr in enumerate(trs):
            t = W.lightcurve_times(name, e)
            A, nfs = event_magnification(tr, t)
            nfs_tot += nfs
            out[f"e{e}"] = A.astype(np.float32 if name == "batched" else np.float64)
        path = W.golden_path(name)
        np.savez_compressed(path, **out)
        print(f"{name}: {len(trs)} events, {sum(a.size for a in out.values())} points, "
              f"{nfs_tot} finite-source points, {time.time() - t0:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["tiny", "large", "sqgrid", "batched"])
