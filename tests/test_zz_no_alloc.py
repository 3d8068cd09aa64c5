"""The allocation-free chi-square/gradient entry point (morse_chi2_grad_noalloc)
against morse_chi2_grad through the C ABI: the same kernels, so the outputs must be
bitwise equal, on two calls in a row (the second smaller: fewer maps, events, points
and candidates, so stale scratch contents would show) and on an oversized request,
which the host rejects with ERANGE before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1511_01157_amd as M
import workloads as W
from paper_1511_01157_amd import _abi
from tests.helpers import note

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def candidates(ev, n, seed):
    tr = ev["truth"]
    rng = np.random.default_rng(seed)
    base = np.array([tr["t0"], tr["u0"], tr["tE"], tr["alpha"]])
    return base + rng.normal(0, 1, (n, 4)) * [0.3 * tr["tE"], 0.05, 0.2 * tr["tE"], 0.2]


def compare(maps, evs, P, ev_idx, map_idx):
    lcs = M.LightCurveBatch.from_events(evs, DEV)
    Pd = torch.from_numpy(P).to(DEV)
    e = torch.from_numpy(np.asarray(ev_idx, np.int32)).to(DEV)
    m = torch.from_numpy(np.asarray(map_idx, np.int32)).to(DEV)
    ref = M.chi2_grad(maps, lcs, Pd, e, m)
    got = M.chi2_grad(maps, lcs, Pd, e, m, noalloc=True)
    torch.cuda.synchronize()
    for a, b, name in zip(got, ref, ("chi2", "grad", "fs", "fb")):
        assert torch.equal(a, b), name
    assert bool(torch.isfinite(got[0]).all())


def test_noalloc_matches_chi2_grad_on_two_calls():
    c = W.config("tiny")
    note("noalloc: build two 512^2 maps")
    m0 = M.build_map(c["s"], c["q"], c["rays"], c["window"], 0.0, device=DEV)
    m1 = M.build_map(1.3, 2e-2, c["rays"], c["window"], 0.0, device=DEV)
    maps = [(m0, c["window"]), (m1, c["window"])]
    e_tiny = W.load_lightcurve("tiny")
    e_b = W.load_lightcurve("batched", 3)
    rng = np.random.default_rng(21)
    P = np.vstack([candidates(e_tiny, 200, 1), candidates(e_b, 100, 2)])
    ev_idx = [0] * 200 + [1] * 100
    map_idx = rng.integers(0, 2, 300)
    note("noalloc: first call, 2 maps, 2 events, 300 candidates")
    compare(maps, [e_tiny, e_b], P, ev_idx, map_idx)
    # second call: one map, one shorter event, fewer candidates
    short = dict(e_tiny)
    for k in ("t", "tt", "F", "sigma", "w"):
        short[k] = e_tiny[k][::3]
    note("noalloc: second call, 1 map, 1 event, 40 candidates")
    compare([(m1, c["window"])], [short], candidates(short, 40, 3), [0] * 40, [0] * 40)


def test_noalloc_rejects_oversized_scratch():
    """Ten 2048^2 maps need 10 x 64 MiB of packed cells, past the 128 MiB array; the
    host returns ERANGE before touching the device (the map pointers are never read)."""
    ctx = M.Context.get(0)
    ev = W.load_lightcurve("tiny")
    lcs = M.LightCurveBatch.from_events([ev], DEV)
    dummy = torch.zeros(4, dtype=torch.float32, device=DEV)
    win = (0.0, 0.0, 3.0, 3.0, 2048, 2048)
    views = (_abi.MapView * 10)(*[_abi.MapView(dummy.data_ptr(), _abi.Grid2D(*win)) for _ in range(10)])
    lca = lcs.abi()
    rc = ctx.lib.morse_chi2_grad_noalloc(ctx.handle, views, 10, ctypes.byref(lca), 0, None, None,
                                         None, None, None, None, None)
    assert rc == _abi.MORSE_ERANGE
    assert b"holds 128 MiB" in ctx.lib.morse_last_error(ctx.handle)
