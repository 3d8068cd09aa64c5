"""Pins of the oracle's L-BFGS state machine (oracle.lbfgs) against things it does not
share code with: a dense BFGS inverse-Hessian recursion (Nocedal & Wright, Numerical
Optimization, eq. 6.17 and alg. 7.4), a hand-derived double-well objective whose first
accepted step has negative curvature, and the Armijo rule checked on the trace.

The refinement's own fixed choices (m stored pairs, H0 = gamma I from the newest pair,
curvature skip s.y <= 1e-12 |s||y|, Armijo c1 with halving, steepest-descent restart)
are restated here in matrix form; each plausible slip in the two-loop code (gamma from
the oldest pair, no history cap, no curvature skip, a wrong shrink or c1) changes at
least one direction or accepted step of the traces below.
"""
import math

import numpy as np
import pytest

from oracle.lbfgs import LbfgsOptions, minimize, store_pair, two_loop_direction

THRESH = 1e-12


def dense_direction(pairs, g):
    """-H g with H from the dense BFGS recursion over the pairs, oldest first:
    H0 = (s.y / y.y) I of the newest pair (1e-2/|g| I without pairs), then
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T."""
    g = np.asarray(g, dtype=np.float64)
    if not pairs:
        return -(1e-2 / np.linalg.norm(g)) * g
    s_n, y_n = pairs[-1]
    H = (s_n @ y_n) / (y_n @ y_n) * np.eye(4)
    for s, y in pairs:
        rho = 1.0 / (s @ y)
        V = np.eye(4) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return -H @ g


def random_pairs(rng, n):
    pairs = []
    while len(pairs) < n:
        s = rng.normal(size=4) * rng.uniform(0.01, 2.0)
        y = rng.normal(size=4) * rng.uniform(0.01, 2.0)
        if s @ y > 0.1 * np.linalg.norm(s) * np.linalg.norm(y):
            pairs.append((s, y))
    return pairs


@pytest.mark.parametrize("n", [0, 1, 2, 5, 8])
def test_two_loop_equals_dense_bfgs(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(25):
        pairs = random_pairs(rng, n)
        g = rng.normal(size=4)
        S = [list(s) for s, _ in pairs]
        Y = [list(y) for _, y in pairs]
        R = [1.0 / float(s @ y) for s, y in pairs]
        d = np.array(two_loop_direction(S, Y, R, list(g)))
        ref = dense_direction(pairs, g)
        assert np.abs(d - ref).max() <= 1e-12 * np.abs(ref).max()


def test_store_pair_caps_history_and_skips_flat_curvature():
    rng = np.random.default_rng(7)
    S, Y, R = [], [], []
    kept = []
    for i in range(13):
        s, y = random_pairs(rng, 1)[0]
        assert store_pair(S, Y, R, list(s), list(y), 8)
        kept.append((s, y))
        assert len(S) == len(Y) == len(R) == min(i + 1, 8)
        for (ks, ky), ss, yy, rr in zip(kept[-8:], S, Y, R):
            assert ss == list(ks) and yy == list(ky)
            assert abs(rr * float(ks @ ky) - 1.0) < 1e-14
    before = [list(v) for v in S]
    s = np.array([1.0, 0.0, 0.0, 0.0])
    for y in ([-1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0], [5e-13, 1.0, 0.0, 0.0]):
        assert not store_pair(S, Y, R, list(s), y, 8)      # s.y <= 1e-12 |s||y|
    assert [list(v) for v in S] == before
    assert store_pair(S, Y, R, list(s), [2e-12, 1.0, 0.0, 0.0], 8)  # just above


def _fl32(v):
    return float(np.float32(v))


def check_trace(trace, objective, opt):
    """Replays a trace of minimize() with the dense model; returns counts of
    (accepted steps, skipped pairs, steps taken with a full history)."""
    pairs = []
    n_skip = n_full = 0
    for k, e in enumerate(trace):
        g = np.array(e["g"])
        d = dense_direction(pairs, g)
        if not g @ d < 0:                              # restart along -g
            pairs = []
            d = dense_direction(pairs, g)
        assert e["pairs"] == len(pairs)
        assert np.abs(np.array(e["d"]) - d).max() <= 1e-9 * np.abs(d).max()
        n_full += len(pairs) == opt.history
        if k + 1 == len(trace):
            break
        # the next accepted point: the first t = shrink^j, j < max_ls, passing Armijo
        p, f, nxt = np.array(e["p"]), e["f"], trace[k + 1]
        gd = float(g @ np.array(e["d"]))
        for j in range(opt.max_ls):
            t = opt.shrink ** j
            pt = np.array([_fl32(p[i] + t * e["d"][i]) for i in range(4)])
            ft, _ = objective(pt)
            if ft <= f + opt.c1 * t * gd:
                break
        else:
            raise AssertionError("no accepted trial before max_ls")
        assert np.array_equal(pt, np.array(nxt["p"])) and ft == nxt["f"]
        s = np.array(nxt["p"]) - p
        y = np.array(nxt["g"]) - g
        if s @ y > THRESH * np.linalg.norm(s) * np.linalg.norm(y):
            pairs = (pairs + [(s, y)])[-opt.history:]
        else:
            n_skip += 1
    return len(trace) - 1, n_skip, n_full


def quadratic():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    A = Q @ np.diag([1.0, 4.0, 25.0, 100.0]) @ Q.T
    b = A @ np.array([0.3, -0.2, 0.1, 0.25])

    def f(p):
        p = np.asarray(p, dtype=np.float64)
        return float(0.5 * p @ A @ p - b @ p), list(A @ p - b)
    return f


def double_well():
    """f = -x0^2/2 + x0^4/4 + (x1^2 + 2 x2^2 + 3 x3^2)/2 at x = p + c: p = 0 sits on the
    concave side of the x0 well (x0 = 0.05) with nearly flat other directions, so the
    first step moves downhill along x0 with s.y < 0."""
    c = np.array([0.05, 1e-3, -1e-3, 1e-3])

    def f(p):
        x = np.asarray(p, dtype=np.float64) + c
        val = -0.5 * x[0] ** 2 + 0.25 * x[0] ** 4 + 0.5 * (x[1] ** 2 + 2 * x[2] ** 2 + 3 * x[3] ** 2)
        return float(val), [-x[0] + x[0] ** 3, x[1], 2 * x[2], 3 * x[3]]
    return f


def test_state_machine_matches_dense_model_on_a_quadratic():
    obj = quadratic()
    opt = LbfgsOptions(steps=60, history=3)
    trace = []
    p, f, fs = minimize(obj, opt, trace)
    accepted, skipped, full = check_trace(trace, obj, opt)
    assert accepted >= opt.history + 3 and full >= 3      # the cap is exercised
    assert all(b <= a for a, b in zip(fs, fs[1:]))
    assert np.abs(np.array([float(v) for v in p]) - np.array([0.3, -0.2, 0.1, 0.25])).max() < 1e-5


def test_state_machine_skips_negative_curvature_pairs():
    obj = double_well()
    opt = LbfgsOptions(steps=200, history=8)
    trace = []
    p, f, fs = minimize(obj, opt, trace)
    accepted, skipped, _ = check_trace(trace, obj, opt)
    assert skipped >= 10 and trace[1]["pairs"] == 0         # concave side: s.y < 0
    assert max(e["pairs"] for e in trace) >= 2              # convex side: pairs kept
    assert abs(float(p[0]) + 0.05 - 1.0) < 1e-3             # rolled into the x0 = 1 well
    assert all(b <= a for a, b in zip(fs, fs[1:]))


def test_noise_free_refinement_recovers_truth_to_1e3():
    from tests.test_oracle_adjoint import WIN, data, smooth_map
    from oracle.lbfgs import refine_one
    amap = smooth_map()
    truth = np.array([0.0, 0.1, 20.0, 0.6])
    t, tt, F, w = data(amap, truth, noise=False)
    for off in ([0.4, 0.01, 0.8, 0.03], [-0.6, -0.008, -1.0, -0.02]):
        p, f, fs = refine_one(amap, WIN, tt, F, w, 0.0, truth + np.array(off), LbfgsOptions(steps=80))
        assert np.abs(p - truth).max() < 1e-3, (off, p - truth)
        assert f < 1e-6 * fs[0]
