"""Precision of the one-pass chi-square on long light curves and near-perfect fits.

A 20000-point light curve (the longest events of the batched workload) whose flux is
the model itself plus noise at 1e-3 of its stated sigma: chi2 is about 1e-6 of the
number of points while V = sum w (F - Fbar)^2 is about 1e3 per point, so the one-pass
form V - F_s C cancels nine digits.  The library's worst-case error bound must send
these trajectories to the direct (compensated) second pass; chi2 and F_s, F_b are
gated at 1e-6 relative against the oracle's two-pass FP64 fit on the same binary32
samples, the gradient at Gate-G against the oracle's FP64 adjoint.
"""
import numpy as np
import pytest
import torch

import paper_1511_01157_amd as M
import workloads as W
from oracle.adjoint import chi2_grad as oracle_grad
from oracle.sampling import sample_mirror32, traj_constants32
from oracle.search import search_mirror32
from tests.helpers import note, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def near_perfect_event(amap, window, n=20000, seed=5):
    rng = np.random.default_rng(seed)
    truth = np.array([0.0, 0.05, 20.0, 0.6])
    tt = np.sort(rng.uniform(-40.0, 40.0, n)).astype(np.float32)
    A = sample_mirror32(amap, window, traj_constants32(truth[None, :], 0.0), tt)[0].astype(np.float64)
    Ft = 1.0 * A + 0.2
    sig = 0.01 * Ft
    F = Ft + 1e-3 * sig * rng.standard_normal(n)
    return {"tt": tt, "F": F, "w": 1.0 / sig ** 2, "t_ref": 0.0}, truth


def test_near_perfect_fit_on_a_long_light_curve(tiny_oracle_map):
    c = W.config("tiny")
    _, _, amap = tiny_oracle_map
    win = c["window"]
    ev, truth = near_perfect_event(amap, win)
    rng = np.random.default_rng(6)
    # the truth, tiny offsets (still near-perfect) and ordinary offsets
    P = np.vstack([truth,
                   truth + rng.normal(0, 1, (7, 4)) * [1e-4, 1e-6, 1e-4, 1e-6],
                   truth + rng.normal(0, 1, (8, 4)) * [0.5, 0.01, 0.5, 0.02]])
    chi2, fs, fb, _ = search_mirror32(amap, win, ev["tt"], ev["F"], ev["w"], P, 0.0)
    V = float(np.sum(ev["w"] * (ev["F"] - np.sum(ev["w"] * ev["F"]) / np.sum(ev["w"])) ** 2))
    assert V / chi2[0] > 1e8          # the cancellation the bound has to catch
    lcs = M.LightCurveBatch.from_events([ev], DEV)
    dm = torch.from_numpy(np.ascontiguousarray(amap, np.float32)).to(DEV)
    tr = M.list_trajectories(torch.from_numpy(P).to(DEV))
    for mode in ("plain", "batched"):
        note(f"precision near-perfect 20000 points search {mode}")
        r = M.search([(dm, win)], lcs, tr, mode, fs=True, fb=True)
        assert rel_err(r["chi2"].cpu().numpy()[0, 0], chi2).max() < 1e-6
        assert rel_err(r["fs"].cpu().numpy()[0, 0], fs, 1e-3).max() < 1e-8
        assert rel_err(r["fb"].cpu().numpy()[0, 0], fb, 1e-3).max() < 1e-8
    note("precision near-perfect 20000 points chi2_grad")
    z = torch.zeros(len(P), dtype=torch.int32, device=DEV)
    gc, gg, _, _ = M.chi2_grad([(dm, win)], lcs, torch.from_numpy(P).to(DEV), z, z)
    oc, og, _, _ = oracle_grad(amap, win, ev["tt"], ev["F"], ev["w"], P, 0.0)
    assert rel_err(gc.cpu().numpy(), oc).max() < 1e-6
    tol = 1e-4 * np.maximum(np.abs(og), 1e-3 * np.abs(og).max(axis=1, keepdims=True))
    assert np.all(np.abs(gg.cpu().numpy() - og) <= tol)
