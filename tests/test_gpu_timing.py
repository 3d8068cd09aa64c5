"""Kernel timing through the C ABI: timed runs launch the same kernels one by one
(results bitwise equal to the graph-replayed runs), count one event pair per launch
of each timed family, and report positive durations."""
import numpy as np
import pytest
import torch

import paper_1511_01157_amd as M
import workloads as W
from tests.helpers import note

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dmap(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def test_timed_runs_match_untimed_and_count_launches(tiny_oracle_map):
    c = W.config("tiny")
    amap = dmap(tiny_oracle_map[2])
    ev = W.load_lightcurve("tiny")
    lcs = M.LightCurveBatch.from_events([ev], DEV)
    trajs = M.grid_trajectories(*W.grid_axes("tiny"))
    maps = [(amap, c["window"])]
    counts = torch.empty((c["window"][5], c["window"][4]), dtype=torch.int32, device=DEV)
    rng = np.random.default_rng(7)
    tr = ev["truth"]
    P = np.array([tr["t0"], tr["u0"], tr["tE"], tr["alpha"]]) + rng.normal(
        0, 1, (16, 4)) * np.array([0.5, 0.01, 1.0, 0.02])
    P = torch.from_numpy(P).to(DEV)
    zeros = torch.zeros(16, dtype=torch.int32, device=DEV)

    def run():
        M.rayshoot(c["s"], c["q"], c["rays"], c["window"], counts)
        r = M.search(maps, lcs, trajs, "batched", top_k=8)
        out, chi2, chi2_0 = M.refine(maps, lcs, P, zeros, zeros, steps=5)
        torch.cuda.synchronize()
        return counts.clone(), r["chi2"].clone(), r["topk_idx"].clone(), out, chi2

    note("timing: untimed reference run")
    ref = run()
    ctx = M.Context.get(0)
    for k in (M.KERNEL_RAYSHOOT, M.KERNEL_SEARCH, M.KERNEL_GRADIENT):
        ctx.kernel_time(k, reset=True)
    note("timing: timed run, all families")
    ctx.set_timing([M.KERNEL_RAYSHOOT, M.KERNEL_SEARCH, M.KERNEL_GRADIENT])
    try:
        got = run()
    finally:
        ctx.set_timing([])
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    launches = {k: ctx.kernel_time(k) for k in (M.KERNEL_RAYSHOOT, M.KERNEL_SEARCH, M.KERNEL_GRADIENT)}
    assert launches[M.KERNEL_RAYSHOOT][1] == 1
    assert launches[M.KERNEL_SEARCH][1] == 1
    assert launches[M.KERNEL_GRADIENT][1] == 6
    for ms, n in launches.values():
        assert ms > 0.0
    # untimed again: nothing more is counted, and reset clears the totals
    run()
    for k in launches:
        assert ctx.kernel_time(k, reset=True)[1] == launches[k][1]
        assert ctx.kernel_time(k) == (0.0, 0)
    with pytest.raises(M.MorseError):
        ctx.kernel_time(3)
    with pytest.raises(M.MorseError):
        ctx.set_timing([5])
