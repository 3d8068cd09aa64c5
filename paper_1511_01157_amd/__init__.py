"""Python binding of the gfx950 MORSE map-build / trajectory-search library.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libmorse.so`` (C ABI in ``include/morse.h``).  PyTorch provides device memory and
streams.  There is no CPU fallback; importing works without a GPU, calling does not.

Entry points (same names as the C ABI):
  build_map(s, q, rays, window, rho)        ray-shooting magnification map (float32)
  rayshoot / normalize_convolve             the two stages of build_map
  search(maps, lcs, trajs, mode)            chi-square of every trajectory on every map
  autotune(maps, lcs, trajs)                pick the batched-search tile shape
  chi2_grad(maps, lcs, params, ev, mi)      chi-square and its gradient
  refine(maps, lcs, params, ev, mi)         batched L-BFGS refinement
  Chi2Fn                                    torch.autograd.Function over chi2_grad
  convolve_stack(counts, rays, window, rhos, gamma)
                                            finite-source maps of several radii
                                            (limb-darkened profile) from one count map
  profile_weights(rho, dx, dy, gamma)       the pixel weights it uses (host)
  caustics(s, q) / caustic_lines(c, r, phi) caustic centres and sizes, (r, phi) lines (host)
  line_filter(map, window, lines, a_min)    minimum-magnification filter of the lines
  lines_to_trajectories(lines, kept, t0, tE) trajectory list of the kept lines
  line_simplex(maps, lcs, lines, start)     downhill simplex over (t0', ln tE) per line and map
Grids are tuples (cx, cy, wx, wy, nx, ny).

A caustic-centred search, for example:
  c = caustics(s, q); L = torch.from_numpy(caustic_lines(c, r, phi)).cuda()
  best, keep, kept = line_filter(amap, window, L, a_min)
  P = lines_to_trajectories(L, kept, t0, tE)
  res = search([(amap, window)], lcs, list_trajectories(P), "batched", top_k=k)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi
from ._abi import (FsOpts, Grid2D, LbfgsOpts, LightCurves, MapStats, MapView, SearchOut, Trajectories,
                   SEARCH_BATCHED, SEARCH_PLAIN, TRAJ_GRID, TRAJ_LIST)

__all__ = ["MorseError", "Context", "LightCurveBatch", "build_map", "rayshoot",
           "normalize_convolve", "convolve_stack", "profile_weights", "caustics", "caustic_lines",
           "fs_magnification", "trajectory_positions", "line_filter", "line_peaks", "peak_starts", "lines_to_trajectories", "line_simplex", "search", "autotune", "autotune_load", "candidates_from_topk", "chi2_grad", "refine", "Chi2Fn",
           "grid_trajectories", "list_trajectories", "abi_version", "KERNEL_RAYSHOOT",
           "KERNEL_SEARCH", "KERNEL_GRADIENT"]

# kernel families of Context.set_timing / Context.kernel_time
KERNEL_RAYSHOOT, KERNEL_SEARCH, KERNEL_GRADIENT = 0, 1, 2


class MorseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"morse error {code}: {msg}")
        self.code = code


def abi_version() -> int:
    return _abi.load().morse_abi_version()


def _grid(g) -> Grid2D:
    cx, cy, wx, wy, nx, ny = g
    return Grid2D(float(cx), float(cy), float(wx), float(wy), int(nx), int(ny))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context per device, enqueuing on torch's current stream."""

    _by_device: dict = {}

    def __init__(self, device: int):
        lib = _abi.load()
        self.device = device
        handle = ctypes.c_void_p()
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib.morse_ctx_create(device, ctypes.c_void_p(stream or None), ctypes.byref(handle))
        if rc != 0:
            raise MorseError(rc, lib.morse_last_error(None).decode())
        self.handle = handle
        self.stream = stream
        self.lib = lib

    @classmethod
    def get(cls, device) -> "Context":
        """The device's shared context, enqueuing on torch's current stream."""
        dev = torch.device(device).index if not isinstance(device, int) else device
        dev = torch.cuda.current_device() if dev is None else dev
        ctx = cls._by_device.get(dev)
        if ctx is None:
            ctx = cls._by_device[dev] = Context(dev)
        ctx.follow_stream()
        return ctx

    @classmethod
    def bound(cls, stream: torch.cuda.Stream) -> "Context":
        """A context of its own (workspace, graphs, metadata) that always enqueues on
        `stream`: pass it as ``ctx=`` to run work concurrently with another context."""
        with torch.cuda.stream(stream):
            ctx = Context(stream.device.index)
        ctx._bound = True
        return ctx

    def follow_stream(self):
        if getattr(self, "_bound", False):
            return
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self.stream:
            self.check(self.lib.morse_ctx_set_stream(self.handle, ctypes.c_void_p(s or None)))
            self.stream = s

    def check(self, rc):
        if rc != 0:
            raise MorseError(rc, self.lib.morse_last_error(self.handle).decode())

    def synchronize(self):
        self.check(self.lib.morse_ctx_synchronize(self.handle))

    def set_timing(self, kernels=()):
        """Bracket every launch of the given kernel families with HIP events on the
        context's stream (an empty set disables timing)."""
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
        self.check(self.lib.morse_ctx_set_timing(self.handle, mask))

    def kernel_time(self, kernel, reset=False):
        """(total ms, launches) of one timed kernel family since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(self.lib.morse_ctx_kernel_time(self.handle, int(kernel), ctypes.byref(ms),
                                                  ctypes.byref(n), int(bool(reset))))
        return ms.value, n.value


def _device_of(t):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.device.index


# ----------------------------------------------------------------------------- maps
def rayshoot(s, q, rays, window, counts, rows=None, accumulate=False, stats=None, ctx=None):
    """Ray counts of lattice rows ``rows`` (default all) into ``counts`` (uint32 as int32)."""
    ctx = ctx or Context.get(_device_of(counts))
    r0, r1 = rows if rows is not None else (0, int(rays[5]))
    ctx.check(ctx.lib.morse_rayshoot(ctx.handle, float(s), float(q), ctypes.byref(_grid(rays)),
                                     ctypes.byref(_grid(window)), int(r0), int(r1), _ptr(counts),
                                     int(bool(accumulate)), _ptr(stats)))
    return counts


def normalize_convolve(counts, rays, window, rho=0.0, out=None, ctx=None):
    ctx = ctx or Context.get(_device_of(counts))
    if out is None:
        out = torch.empty((int(window[5]), int(window[4])), dtype=torch.float32, device=counts.device)
    ctx.check(ctx.lib.morse_normalize_convolve(ctx.handle, _ptr(counts), ctypes.byref(_grid(rays)),
                                               ctypes.byref(_grid(window)), float(rho), _ptr(out)))
    return out


def convolve_stack(counts, rays, window, rhos, gamma=0.53, fft_min_taps=0, out=None, ctx=None):
    """Finite-source maps float32[len(rhos), ny, nx] of one count map for each source
    radius, limb-darkened profile with coefficient gamma (0 = uniform disk)."""
    ctx = ctx or Context.get(_device_of(counts))
    rh = np.ascontiguousarray(np.asarray(rhos, dtype=np.float64).reshape(-1))
    if out is None:
        out = torch.empty((len(rh), int(window[5]), int(window[4])), dtype=torch.float32,
                          device=counts.device)
    ctx.check(ctx.lib.morse_convolve_stack(ctx.handle, _ptr(counts), ctypes.byref(_grid(rays)),
                                           ctypes.byref(_grid(window)), rh.ctypes.data, len(rh),
                                           float(gamma), int(fft_min_taps), _ptr(out)))
    return out


def profile_weights(rho, dx, dy, gamma=0.53):
    """The library's FP64 pixel weights [2ry+1, 2rx+1] of one limb-darkened disk (host)."""
    lib = _abi.load()
    rx, ry = ctypes.c_int32(), ctypes.c_int32()
    rc = lib.morse_profile_weights(float(rho), float(dx), float(dy), float(gamma), None, 0,
                                   ctypes.byref(rx), ctypes.byref(ry))
    if rc != _abi.MORSE_OK:
        raise MorseError(rc, lib.morse_last_error(None).decode())
    w = np.empty((2 * ry.value + 1, 2 * rx.value + 1), dtype=np.float64)
    rc = lib.morse_profile_weights(float(rho), float(dx), float(dy), float(gamma), w.ctypes.data,
                                   w.size, ctypes.byref(rx), ctypes.byref(ry))
    if rc != _abi.MORSE_OK:
        raise MorseError(rc, lib.morse_last_error(None).decode())
    return w


def build_map(s, q, rays, window, rho=0.0, device="cuda", out=None, counts=None, stats=False, ctx=None):
    """Magnification map float32[ny, nx]; with stats=True also a dict of ray statistics."""
    dev = torch.device(device)
    if out is None:
        out = torch.empty((int(window[5]), int(window[4])), dtype=torch.float32, device=dev)
    ctx = ctx or Context.get(_device_of(out))
    st = MapStats() if stats else None
    ctx.check(ctx.lib.morse_build_map(ctx.handle, float(s), float(q), ctypes.byref(_grid(rays)),
                                      ctypes.byref(_grid(window)), float(rho), _ptr(counts),
                                      _ptr(out), ctypes.byref(st) if st is not None else None))
    if stats:
        return out, {k: int(getattr(st, k)) for k, _ in MapStats._fields_ if k != "reserved"}
    return out


# --------------------------------------------------------------------------- search
@dataclass
class LightCurveBatch:
    """Concatenated light curves: device t (float32 offsets), flux, weight (float64)."""
    t: torch.Tensor
    flux: torch.Tensor
    weight: torch.Tensor
    offsets: np.ndarray  # host int64 [n_events + 1]
    t_ref: np.ndarray    # host float64 [n_events]

    @classmethod
    def from_events(cls, events, device="cuda"):
        """events: iterable of dicts with tt (float32 offsets), F, w, t_ref."""
        events = list(events)
        offs = np.zeros(len(events) + 1, dtype=np.int64)
        offs[1:] = np.cumsum([len(e["tt"]) for e in events])
        cat = lambda k, dt: torch.from_numpy(np.concatenate([np.asarray(e[k], dt) for e in events])).to(device)
        return cls(cat("tt", np.float32), cat("F", np.float64), cat("w", np.float64), offs,
                   np.array([e["t_ref"] for e in events], dtype=np.float64))

    @property
    def n_events(self):
        return len(self.t_ref)

    def abi(self):
        self._keep = (np.ascontiguousarray(self.offsets, np.int64), np.ascontiguousarray(self.t_ref, np.float64))
        return LightCurves(self.n_events, 0, self._keep[0].ctypes.data, self._keep[1].ctypes.data,
                           self.t.data_ptr(), self.flux.data_ptr(), self.weight.data_ptr())


class _Trajs:
    def __init__(self, kind, n, axes=None, params=None, shared=True):
        self.kind, self.n, self.axes, self.params, self.shared = kind, n, axes, params, shared

    def abi(self):
        if self.kind == TRAJ_GRID:
            self._keep = [np.ascontiguousarray(a, np.float64) for a in self.axes]
            u, a, t0, te = self._keep
            return Trajectories(TRAJ_GRID, len(u), len(a), len(t0), len(te), 1, u.ctypes.data,
                                a.ctypes.data, t0.ctypes.data, te.ctypes.data, 0, None)
        return Trajectories(TRAJ_LIST, 0, 0, 0, 0, int(self.shared), None, None, None, None,
                            int(self.n), self.params.data_ptr())


def grid_trajectories(u0s, alphas, t0s, tEs):
    """Product grid, index ((iu0 * n_alpha + ia) * n_t0 + it0) * n_tE + itE."""
    axes = [np.asarray(v, np.float64).ravel() for v in (u0s, alphas, t0s, tEs)]
    return _Trajs(TRAJ_GRID, int(np.prod([len(a) for a in axes])), axes=axes)


def list_trajectories(params: torch.Tensor, shared=True):
    """Device float64 rows (t0, u0, tE, alpha): [n, 4] shared, or [n_events, n, 4]."""
    if params.dtype != torch.float64 or not params.is_contiguous():
        raise ValueError("params must be contiguous float64")
    n = params.shape[-2]
    return _Trajs(TRAJ_LIST, n, params=params, shared=shared)


def _map_views(maps):
    views = (MapView * len(maps))()
    for i, (m, w) in enumerate(maps):
        if m.dtype != torch.float32 or not m.is_contiguous() or tuple(m.shape) != (int(w[5]), int(w[4])):
            raise ValueError(f"map {i} must be contiguous float32 [ny, nx] matching its window")
        views[i] = MapView(m.data_ptr(), _grid(w))
    return views


# ----------------------------------------------------- caustic-centred lines + filter
def caustics(s, q, nphi=4096):
    """Separate caustics of the lens (s, q): float64 [n, 5] rows (cx, cy, half_w, half_h, size)."""
    lib = _abi.load()
    n = ctypes.c_int32()
    rc = lib.morse_caustics(float(s), float(q), int(nphi), None, 0, ctypes.byref(n))
    if rc != _abi.MORSE_OK:
        raise MorseError(rc, lib.morse_last_error(None).decode())
    out = np.empty((n.value, 5), dtype=np.float64)
    rc = lib.morse_caustics(float(s), float(q), int(nphi), out.ctypes.data, n.value, ctypes.byref(n))
    if rc != _abi.MORSE_OK:
        raise MorseError(rc, lib.morse_last_error(None).decode())
    return out


def caustic_lines(caus, r, phi):
    """Lines float64 [n_caustics * n_r * n_phi, 3] (u0, alpha, shift), caustic-major."""
    lib = _abi.load()
    c = np.ascontiguousarray(np.asarray(caus, dtype=np.float64).reshape(-1, 5))
    rr = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
    pp = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
    out = np.empty((len(c) * len(rr) * len(pp), 3), dtype=np.float64)
    rc = lib.morse_caustic_lines(c.ctypes.data, len(c), rr.ctypes.data, len(rr), pp.ctypes.data,
                                 len(pp), out.ctypes.data)
    if rc != _abi.MORSE_OK:
        raise MorseError(rc, lib.morse_last_error(None).decode())
    return out


def line_filter(amap, window, lines, a_min, ctx=None):
    """Minimum-magnification filter of device lines float64 [n, 3] on one map:
    (best float32 [n], keep uint8 [n], kept int64 [count] ascending)."""
    ctx = ctx or Context.get(_device_of(amap))
    if lines.dtype != torch.float64 or not lines.is_contiguous() or lines.shape[-1] != 3:
        raise ValueError("lines must be contiguous float64 [n, 3]")
    n = lines.shape[0]
    best = torch.empty(n, dtype=torch.float32, device=lines.device)
    keep = torch.empty(n, dtype=torch.uint8, device=lines.device)
    kept = torch.empty(max(n, 1), dtype=torch.int64, device=lines.device)
    count = ctypes.c_int64()
    view = MapView(amap.data_ptr(), _grid(window))
    ctx.check(ctx.lib.morse_line_filter(ctx.handle, ctypes.byref(view), _ptr(lines), n, float(a_min),
                                        _ptr(best), _ptr(keep), _ptr(kept), None, ctypes.byref(count)))
    return best, keep, kept[:count.value]


def line_peaks(amap, window, lines, a_min, min_peaks=0, hysteresis=0.0, max_peaks=8, ctx=None):
    """Peak library of device lines float64 [n, 3] on one map, with the rejection of
    lines below a_min or with fewer than min_peaks peaks: (best float32 [n], npeaks int32
    [n], peak_tau float32 [n, max_peaks], peak_A float32 [n, max_peaks], keep uint8 [n],
    kept int64 [count] ascending)."""
    ctx = ctx or Context.get(_device_of(amap))
    if lines.dtype != torch.float64 or not lines.is_contiguous() or lines.shape[-1] != 3:
        raise ValueError("lines must be contiguous float64 [n, 3]")
    n = lines.shape[0]
    dev = lines.device
    best = torch.empty(n, dtype=torch.float32, device=dev)
    npk = torch.empty(n, dtype=torch.int32, device=dev)
    ptau = torch.empty((n, max_peaks), dtype=torch.float32, device=dev)
    pA = torch.empty((n, max_peaks), dtype=torch.float32, device=dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    kept = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    count = ctypes.c_int64()
    view = MapView(amap.data_ptr(), _grid(window))
    ctx.check(ctx.lib.morse_line_peaks(ctx.handle, ctypes.byref(view), _ptr(lines), n, float(a_min),
                                       int(min_peaks), float(hysteresis), int(max_peaks), _ptr(best),
                                       _ptr(npk), _ptr(ptau), _ptr(pA), _ptr(keep), _ptr(kept), None,
                                       ctypes.byref(count)))
    return best, npk, ptau, pA, keep, kept[:count.value]


def peak_starts(lines, kept, npeaks, peak_tau, peak_A, tp, tE=0.0, ctx=None):
    """Simplex starts float64 [len(kept), 2] (t0', tE) from one or two observed peak
    times tp (Eqs. 7-8); ``kept`` None means every line."""
    ctx = ctx or Context.get(_device_of(lines))
    tp = np.ascontiguousarray(np.atleast_1d(tp), dtype=np.float64)
    n = lines.shape[0] if kept is None else kept.shape[0]
    start = torch.empty((n, 2), dtype=torch.float64, device=lines.device)
    ctx.check(ctx.lib.morse_peak_starts(ctx.handle, _ptr(lines), _ptr(kept) if kept is not None else None,
                                        n, _ptr(npeaks), _ptr(peak_tau), _ptr(peak_A),
                                        int(peak_tau.shape[1]), tp.ctypes.data, len(tp), float(tE),
                                        _ptr(start)))
    return start


def lines_to_trajectories(lines, kept, t0, tE, ctx=None):
    """Trajectory rows float64 [n_kept * n_t0 * n_tE, 4] (t0, u0, tE, alpha) of the kept
    lines (all lines when kept is None); t0 = time of closest approach to the caustic centre."""
    ctx = ctx or Context.get(_device_of(lines))
    a = np.ascontiguousarray(np.asarray(t0, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(tE, dtype=np.float64).reshape(-1))
    nk = lines.shape[0] if kept is None else kept.shape[0]
    out = torch.empty((nk * len(a) * len(b), 4), dtype=torch.float64, device=lines.device)
    ctx.check(ctx.lib.morse_lines_to_trajectories(ctx.handle, _ptr(lines), _ptr(kept), nk,
                                                  a.ctypes.data, len(a), b.ctypes.data, len(b),
                                                  _ptr(out)))
    return out


def line_simplex(maps, lcs: LightCurveBatch, lines, start, event=0, max_iter=5000, step_t0=2.0,
                 step_ln_tE=0.2, ftol=1e-10, ctx=None):
    """Downhill simplex over (t0', ln tE) of every device line [n, 3] on every map, from
    start [n, 2] (t0', tE): (chi2, t0', tE, iterations, evaluations), each [n, n_maps]."""
    ctx = ctx or Context.get(_device_of(lines))
    views = _map_views(maps)
    for t, k in ((lines, 3), (start, 2)):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.shape[-1] != k:
            raise ValueError("lines [n, 3] and start [n, 2] must be contiguous float64")
    n = lines.shape[0]
    shape = (n, len(maps))
    chi2 = torch.empty(shape, dtype=torch.float64, device=lines.device)
    t0 = torch.empty(shape, dtype=torch.float64, device=lines.device)
    tE = torch.empty(shape, dtype=torch.float64, device=lines.device)
    it = torch.empty(shape, dtype=torch.int32, device=lines.device)
    ev = torch.empty(shape, dtype=torch.int32, device=lines.device)
    opts = _abi.SimplexOpts(int(max_iter), 0, float(step_t0), float(step_ln_tE), float(ftol))
    lc = lcs.abi()
    ctx.check(ctx.lib.morse_line_simplex(ctx.handle, views, len(maps), ctypes.byref(lc), int(event),
                                         _ptr(lines), n, _ptr(start), ctypes.byref(opts), _ptr(chi2),
                                         _ptr(t0), _ptr(tE), _ptr(it), _ptr(ev)))
    return chi2, t0, tE, it, ev


def search(maps, lcs: LightCurveBatch, trajs, mode="plain", chi2=True, fs=False, fb=False,
           best=False, top_k=0, out=None, ctx=None):
    """Chi-square of every trajectory on every map for every event.

    maps: list of (map tensor, window).  Returns a dict with the requested outputs:
    chi2/fs/fb [n_events, n_maps, n_traj], best_chi2/best_idx [n_events, n_maps],
    topk_chi2/topk_idx [n_events, top_k] (index = map * n_traj + traj).  ``out`` (a
    dict from an earlier call with the same arguments) is reused instead of allocating;
    the batched mode replays its captured graph only when all buffers are the same.
    """
    dev = lcs.t.device
    ctx = ctx or Context.get(_device_of(lcs.t))
    ne, nm, nt = lcs.n_events, len(maps), trajs.n
    want = {"chi2": ((ne, nm, nt), torch.float64) if chi2 else None,
            "fs": ((ne, nm, nt), torch.float64) if fs else None,
            "fb": ((ne, nm, nt), torch.float64) if fb else None,
            "best_chi2": ((ne, nm), torch.float64) if best else None,
            "best_idx": ((ne, nm), torch.int64) if best else None,
            "topk_chi2": ((ne, top_k), torch.float64) if top_k else None,
            "topk_idx": ((ne, top_k), torch.int64) if top_k else None}
    res = {}
    for k, spec in want.items():
        if spec is None:
            continue
        shape, dt = spec
        t = out.get(k) if out else None
        if t is None or tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous():
            t = torch.empty(shape, dtype=dt, device=dev)
        res[k] = t
    out = SearchOut(*(res[k].data_ptr() if k in res else None
                      for k in ("chi2", "fs", "fb", "best_chi2", "best_idx")),
                    int(top_k), 0, res["topk_chi2"].data_ptr() if top_k else None,
                    res["topk_idx"].data_ptr() if top_k else None)
    views = _map_views(maps)
    lca = lcs.abi()
    ta = trajs.abi()
    m = {"plain": SEARCH_PLAIN, "batched": SEARCH_BATCHED}[mode]
    ctx.check(ctx.lib.morse_search(ctx.handle, views, nm, ctypes.byref(lca), ctypes.byref(ta), m,
                                   ctypes.byref(out)))
    return res


def autotune(maps, lcs: LightCurveBatch, trajs, cache_path=None, ctx=None):
    ctx = ctx or Context.get(_device_of(lcs.t))
    best = ctypes.c_int32(-1)
    views = _map_views(maps)
    lca = lcs.abi()
    ta = trajs.abi()
    ctx.check(ctx.lib.morse_autotune(ctx.handle, views, len(maps), ctypes.byref(lca), ctypes.byref(ta),
                                     cache_path.encode() if cache_path else None, ctypes.byref(best)))
    return best.value


def autotune_load(cache_path, device=0, ctx=None):
    """Take the shapes of an autotune cache file; returns the number of classes loaded."""
    ctx = ctx or Context.get(device)
    n = ctypes.c_int32(0)
    ctx.check(ctx.lib.morse_autotune_load(ctx.handle, str(cache_path).encode(), ctypes.byref(n)))
    return n.value


def candidates_from_topk(trajs, topk_idx, n_maps, out=None, ctx=None):
    """Refinement candidates from a search's top-k: params [n_events*k, 4] float64,
    event and map index [n_events*k] int32 (written into ``out`` when given)."""
    ne, k = topk_idx.shape
    dev = topk_idx.device
    ctx = ctx or Context.get(_device_of(topk_idx))
    if out is not None:
        params, event, mapi = out
    else:
        params = torch.empty((ne * k, 4), dtype=torch.float64, device=dev)
        event = torch.empty(ne * k, dtype=torch.int32, device=dev)
        mapi = torch.empty(ne * k, dtype=torch.int32, device=dev)
    ta = trajs.abi()
    ctx.check(ctx.lib.morse_candidates_from_topk(ctx.handle, ctypes.byref(ta), int(ne), int(n_maps),
                                                 int(k), _ptr(topk_idx.contiguous()), _ptr(params),
                                                 _ptr(event), _ptr(mapi)))
    return params, event, mapi


# --------------------------------------------------- finite-source magnification
def fs_magnification(s, q, zeta, rho, gamma=0.0, n_b=192, n_crit=1024, n_side=128, n_grow=40,
                     n_r=512, n_theta=512, n_shrink=2, near=10.0, gap=0.2, ctx=None):
    """Image-centred ray-shooting magnification of sources at device positions zeta
    float64 [n, 2] (or complex128 [n]): (A float64 [n], regions int32 [n])."""
    if zeta.dtype == torch.complex128:
        zeta = torch.view_as_real(zeta.contiguous())
    if zeta.dtype != torch.float64 or zeta.dim() != 2 or zeta.shape[1] != 2 or not zeta.is_contiguous():
        raise ValueError("zeta must be contiguous float64 [n, 2] or complex128 [n]")
    ctx = ctx or Context.get(_device_of(zeta))
    n = zeta.shape[0]
    A = torch.empty(n, dtype=torch.float64, device=zeta.device)
    nreg = torch.empty(n, dtype=torch.int32, device=zeta.device)
    o = FsOpts(int(n_b), int(n_crit), int(n_side), int(n_grow), int(n_r), int(n_theta), int(n_shrink), 0,
               float(near), float(gap))
    ctx.check(ctx.lib.morse_fs_magnification(ctx.handle, float(s), float(q), _ptr(zeta), n, float(rho),
                                             float(gamma), ctypes.byref(o), _ptr(A), _ptr(nreg)))
    return A, nreg


def trajectory_positions(params, t, ctx=None):
    """Source positions float64 [n, 2] of the trajectory params (t0, u0, tE, alpha) at
    device FP64 times t [n]."""
    if t.dtype != torch.float64 or t.dim() != 1 or not t.is_contiguous():
        raise ValueError("t must be contiguous float64 [n]")
    ctx = ctx or Context.get(_device_of(t))
    p = np.ascontiguousarray(params, dtype=np.float64).reshape(4)
    zeta = torch.empty((t.shape[0], 2), dtype=torch.float64, device=t.device)
    ctx.check(ctx.lib.morse_trajectory_positions(ctx.handle, p.ctypes.data, _ptr(t), t.shape[0],
                                                 _ptr(zeta)))
    return zeta


# ------------------------------------------------------------------ gradient / refine
def _cand_args(params, event, map_index):
    if params.dtype != torch.float64 or params.dim() != 2 or params.shape[1] != 4 or not params.is_contiguous():
        raise ValueError("params must be contiguous float64 [n, 4]")
    n = params.shape[0]
    for name, t in (("event", event), ("map_index", map_index)):
        if t.dtype != torch.int32 or t.shape != (n,) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous int32 [n]")
    return n


def chi2_grad(maps, lcs: LightCurveBatch, params, event, map_index, grad=True, ctx=None,
              noalloc=False):
    """chi2 [n], grad [n, 4] (d/d t0, u0, tE, alpha), Fs [n], Fb [n].  ``noalloc``
    calls the allocation-free entry point (scratch in the library's static array)."""
    n = _cand_args(params, event, map_index)
    ctx = ctx or Context.get(_device_of(params))
    dev = params.device
    chi2 = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty((n, 4), dtype=torch.float64, device=dev) if grad else None
    fs = torch.empty(n, dtype=torch.float64, device=dev)
    fb = torch.empty(n, dtype=torch.float64, device=dev)
    views = _map_views(maps)
    lca = lcs.abi()
    fn = ctx.lib.morse_chi2_grad_noalloc if noalloc else ctx.lib.morse_chi2_grad
    ctx.check(fn(ctx.handle, views, len(maps), ctypes.byref(lca), n, _ptr(params), _ptr(event),
                 _ptr(map_index), _ptr(chi2), _ptr(g), _ptr(fs), _ptr(fb)))
    return chi2, g, fs, fb


def refine(maps, lcs: LightCurveBatch, params, event, map_index, steps=50, history=8, max_ls=10,
           c1=1e-4, shrink=0.5, inplace=False, chi2_out=None, ctx=None):
    """Refined params, final chi2 and initial chi2.  With ``inplace`` the refined
    parameters overwrite ``params``; ``chi2_out`` = (chi2, chi2_init) buffers to reuse
    (the captured rounds replay only when every buffer is the same)."""
    n = _cand_args(params, event, map_index)
    ctx = ctx or Context.get(_device_of(params))
    out = params if inplace else params.clone()
    if chi2_out is not None:
        chi2, chi2_0 = chi2_out
    else:
        chi2 = torch.empty(n, dtype=torch.float64, device=params.device)
        chi2_0 = torch.empty(n, dtype=torch.float64, device=params.device)
    opts = LbfgsOpts(int(steps), int(history), int(max_ls), 0, float(c1), float(shrink))
    views = _map_views(maps)
    lca = lcs.abi()
    ctx.check(ctx.lib.morse_refine(ctx.handle, views, len(maps), ctypes.byref(lca), n, _ptr(out),
                                   _ptr(event), _ptr(map_index), ctypes.byref(opts), _ptr(chi2),
                                   _ptr(chi2_0)))
    return out, chi2, chi2_0


class Chi2Fn(torch.autograd.Function):
    """chi2 = Chi2Fn.apply(params [n, 4] float64, maps, lcs, event, map_index).

    Forward runs the gradient kernel once and saves d chi2 / d params; backward
    returns grad_out[:, None] * saved gradient.
    """

    @staticmethod
    def forward(ctx, params, maps, lcs, event, map_index):
        chi2, g, _, _ = chi2_grad(maps, lcs, params.detach().contiguous(), event, map_index)
        ctx.save_for_backward(g)
        return chi2

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[:, None] * g, None, None, None, None
