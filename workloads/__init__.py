"""Seeded synthetic inputs for the five workloads (shared by tests, oracle and bench).

This module holds the workload definitions and every random draw; it contains none
of the method's arithmetic (no lens equation, no sampling, no fit).  The true
magnification of each light-curve point is computed once by
``tests/golden/make_lightcurves.py`` with the oracle and stored in
``tests/golden/lc_amag_<name>.npz``; ``load_lightcurve`` combines it with the seeded
times and noise deviates into an observed light curve.

Workloads (the five benchmark configurations):
  tiny      s=1, q=1e-3, 3200^2 rays over [-2,2]^2 -> 512^2 map over [-1,1]^2, point
            source; 1000-point light curve, 32 u0 x 32 alpha grid at fixed t0, tE.
  large     s=0.8, q=5e-3, 32768^2 rays over [-3,3]^2 -> 2048^2 map over [-1.5,1.5]^2,
            disk rho=2e-3; 3000 points; 64 u0 x 64 alpha x 16 t0 x 8 tE grid.
  sqgrid    24 s x 16 q = 384 maps, 16384^2 rays over [-3,3]^2 -> 1024^2 over
            [-1.5,1.5]^2, rho=1e-3; 3000 points; 1e5 random trajectories.
  batched   256 events, lognormal lengths (median 2000, sigma_ln 1, clip 200..20000),
            own truths; 64-map bank (8 s x 8 q) at 1024^2, 16384^2 rays, point source;
            32768 random trajectories per event.
  refine    first 64 events of ``batched``; the same 64 (s, q) at 2048^2 with 32768^2
            rays; top 4096 candidates per event, 50 L-BFGS rounds.

Grids are tuples (cx, cy, wx, wy, nx, ny).  Trajectory parameters are rows
(t0, u0, tE, alpha) in FP64.  Product grids are row-major over (u0, alpha, t0, tE).
"""
from __future__ import annotations

import os

import numpy as np

__all__ = ["SEED", "NAMES", "config", "rng", "lightcurve_times", "truths",
           "grid_axes", "random_trajectories", "load_lightcurve", "golden_path",
           "map_bank"]

SEED = 151101157
NAMES = ("tiny", "large", "sqgrid", "batched", "refine")
_IDS = {n: i for i, n in enumerate(NAMES)}
GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden")

# stream ids of the seeded generators
_S_TIMES, _S_GAPS, _S_NOISE, _S_TRUTH, _S_TRAJ, _S_LEN = range(6)


def rng(name: str, stream: int, event: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED, _IDS[name], stream, event]))


def _truth0(rho):
    return dict(t0=0.0, u0=0.05, tE=20.0, alpha=0.6, Fs=1.0, Fb=0.2, rho=rho)


_CFG = {
    "tiny": dict(s=1.0, q=1e-3, rays=(0.0, 0.0, 4.0, 4.0, 3200, 3200),
                 window=(0.0, 0.0, 2.0, 2.0, 512, 512), rho=0.0, npts=1000,
                 truth=_truth0(0.0), lc_rho=0.0),
    "large": dict(s=0.8, q=5e-3, rays=(0.0, 0.0, 6.0, 6.0, 32768, 32768),
                  window=(0.0, 0.0, 3.0, 3.0, 2048, 2048), rho=2e-3, npts=3000,
                  truth=_truth0(2e-3), lc_rho=2e-3),
    "sqgrid": dict(s=0.8, q=5e-3, rays=(0.0, 0.0, 6.0, 6.0, 16384, 16384),
                   window=(0.0, 0.0, 3.0, 3.0, 1024, 1024), rho=1e-3, npts=3000,
                   truth=_truth0(1e-3), lc_rho=1e-3, n_s=24, n_q=16, n_traj=100_000),
    "batched": dict(rays=(0.0, 0.0, 6.0, 6.0, 16384, 16384),
                    window=(0.0, 0.0, 3.0, 3.0, 1024, 1024), rho=0.0, n_events=256,
                    n_s=8, n_q=8, n_traj=32768, median_len=2000, sigma_ln=1.0,
                    len_clip=(200, 20000)),
    "refine": dict(rays=(0.0, 0.0, 6.0, 6.0, 32768, 32768),
                   window=(0.0, 0.0, 3.0, 3.0, 2048, 2048), rho=0.0, n_events=64,
                   top_k=4096, steps=50, history=8, max_ls=10, c1=1e-4, shrink=0.5),
}


def config(name: str) -> dict:
    c = dict(_CFG[name])
    c["name"] = name
    return c


def map_bank(name: str):
    """(s, q) pairs of a multi-map workload, s-major order."""
    if name == "sqgrid":
        c = _CFG[name]
        s = np.logspace(np.log10(0.3), np.log10(3.0), c["n_s"])
        q = np.logspace(-4.0, -1.0, c["n_q"])
    elif name in ("batched", "refine"):
        s = np.logspace(np.log10(0.3), np.log10(3.0), 8)
        q = np.logspace(-4.0, -1.0, 8)
    else:
        c = _CFG[name]
        return np.array([[c["s"], c["q"]]])
    S, Q = np.meshgrid(s, q, indexing="ij")
    return np.stack([S.ravel(), Q.ravel()], axis=1)


def truths(name: str):
    """List of per-event truth dicts (t0, u0, tE, alpha, Fs, Fb, rho, s, q, npts)."""
    if name in ("tiny", "large", "sqgrid"):
        c = _CFG[name]
        tr = dict(c["truth"])
        tr.update(s=c["s"], q=c["q"], npts=c["npts"])
        return [tr]
    c = _CFG["batched"]
    r = rng("batched", _S_TRUTH)
    ln = rng("batched", _S_LEN)
    out = []
    n_ev = c["n_events"]
    lens = np.exp(np.log(c["median_len"]) + c["sigma_ln"] * ln.standard_normal(n_ev))
    lens = np.clip(np.rint(lens), *c["len_clip"]).astype(int)
    for e in range(n_ev):
        out.append(dict(
            s=float(10 ** r.uniform(np.log10(0.3), np.log10(3.0))),
            q=float(10 ** r.uniform(-4.0, -1.0)),
            u0=float(r.uniform(0.001, 0.3)),
            alpha=float(r.uniform(0.0, 2 * np.pi)),
            tE=float(10 ** r.uniform(np.log10(5.0), np.log10(100.0))),
            rho=float(10 ** r.uniform(-4.0, np.log10(5e-3))),
            t0=float(2456000.0 + r.uniform(0.0, 365.0)),
            Fs=1.0, Fb=float(r.uniform(0.0, 1.0)), npts=int(lens[e])))
    if name == "refine":
        return out[: _CFG["refine"]["n_events"]]
    return out


def lightcurve_times(name: str, event: int = 0) -> np.ndarray:
    """Sorted FP64 observation times of one event (i.i.d. uniform, two 1-day gaps; 2-5 gaps of 0.3-3 d for batched)."""
    key = "batched" if name == "refine" else name
    tr = truths(key)[event]
    lo, hi = tr["t0"] - 2 * tr["tE"], tr["t0"] + 2 * tr["tE"]
    rg = rng(key, _S_GAPS, event)
    if key == "batched":
        ngap = int(rg.integers(2, 6))
        glen = rg.uniform(0.3, 3.0, ngap)
    else:
        ngap = 2
        glen = np.ones(2)
    gs = rg.uniform(lo, hi - glen)
    rt = rng(key, _S_TIMES, event)
    n = tr["npts"]
    kept = np.empty(0)
    while kept.size < n:
        t = rt.uniform(lo, hi, 2 * n)
        bad = np.zeros(t.size, bool)
        for g0, gl in zip(gs, glen):
            bad |= (t >= g0) & (t < g0 + gl)
        kept = np.concatenate([kept, t[~bad]])
    return np.sort(kept[:n])


def noise_deviates(name: str, n: int, event: int = 0) -> np.ndarray:
    key = "batched" if name == "refine" else name
    return rng(key, _S_NOISE, event).standard_normal(n)


def grid_axes(name: str):
    """(u0s, alphas, t0s, tEs) of a product-grid workload (u0 log-spaced, alpha = 2 pi k / n, t0 linear over t0 +- tE/2, tE log-spaced 5..100)."""
    tr = truths(name)[0]
    if name == "tiny":
        return (np.logspace(-3, np.log10(0.5), 32), 2 * np.pi * np.arange(32) / 32,
                np.array([tr["t0"]]), np.array([tr["tE"]]))
    if name == "large":
        return (np.logspace(-3, np.log10(0.5), 64), 2 * np.pi * np.arange(64) / 64,
                np.linspace(tr["t0"] - 0.5 * tr["tE"], tr["t0"] + 0.5 * tr["tE"], 16),
                np.logspace(np.log10(5.0), np.log10(100.0), 8))
    raise KeyError(name)


def random_trajectories(name: str, event: int = 0, n: int | None = None) -> np.ndarray:
    """Uniform draws over (u0 in [0, 0.5), alpha, t0 +- 0.5 tE, log-uniform tE 5..100)."""
    key = "batched" if name == "refine" else name
    tr = truths(key)[event]
    n = n or _CFG[key]["n_traj"]
    r = rng(key, _S_TRAJ, event)
    u0 = r.uniform(0.0, 0.5, n)
    al = r.uniform(0.0, 2 * np.pi, n)
    t0 = tr["t0"] + r.uniform(-0.5, 0.5, n) * tr["tE"]
    tE = 10 ** r.uniform(np.log10(5.0), np.log10(100.0), n)
    return np.stack([t0, u0, tE, al], axis=1)


def golden_path(name: str) -> str:
    key = "batched" if name == "refine" else name
    return os.path.join(GOLDEN, f"lc_amag_{key}.npz")


def load_lightcurve(name: str, event: int = 0):
    """Observed light curve of one event: dict(t, tt, t_ref, F, sigma, w, truth).

    F_true = Fs A_true + Fb (Eq. 5 as the observation model), sigma = 1% of F_true,
    F = F_true + sigma * N(0, 1), w = 1/sigma^2, t_ref the mid-time, and
    tt = fl32(t - t_ref) the FP32 time offsets the search consumes.
    """
    key = "batched" if name == "refine" else name
    tr = truths(key)[event]
    t = lightcurve_times(key, event)
    with np.load(golden_path(key)) as z:
        amag = np.asarray(z[f"e{event}"], dtype=np.float64)
    if amag.shape != t.shape:
        raise ValueError(f"stored magnifications do not match {key} event {event}")
    Ftrue = tr["Fs"] * amag + tr["Fb"]
    sigma = 0.01 * Ftrue
    F = Ftrue + sigma * noise_deviates(key, t.size, event)
    t_ref = 0.5 * (t[0] + t[-1])
    return dict(t=t, tt=(t - t_ref).astype(np.float32), t_ref=t_ref, F=F, sigma=sigma,
                w=1.0 / (sigma * sigma), truth=tr)
