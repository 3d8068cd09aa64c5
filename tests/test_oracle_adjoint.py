"""Pins of oracle.adjoint (envelope gradient) and oracle.lbfgs (refinement)."""
import numpy as np
import pytest

from oracle.adjoint import chi2_grad, chi2_grad_explicit, fd_gradient
from oracle.lbfgs import LbfgsOptions, refine, refine_one
from oracle.lens import paczynski
from oracle.sampling import sample_mirror32, traj_constants32

WIN = (0.0, 0.0, 2.0, 2.0, 256, 256)


def smooth_map():
    """A smooth asymmetric test map: Paczynski about the origin plus a Gaussian bump."""
    d = 2.0 / 256
    c = -1 + (np.arange(256) + 0.5) * d
    X, Y = np.meshgrid(c, c)
    return (paczynski(np.hypot(X, Y) + 0.05) + 2.0 * np.exp(-((X - 0.2) ** 2 + (Y - 0.25) ** 2) / 0.02)
            ).astype(np.float32)


def data(amap, truth, n=300, seed=0, noise=True):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(-40, 40, n))
    tt = t.astype(np.float32)
    A = sample_mirror32(amap, WIN, traj_constants32(truth[None, :], 0.0), tt)[0].astype(float)
    Ftrue = 1.0 * A + 0.2
    sig = 0.01 * Ftrue
    F = Ftrue + (sig * rng.standard_normal(n) if noise else 0.0)
    return t, tt, F, 1 / sig ** 2


def test_envelope_equals_explicit_solve():
    amap = smooth_map()
    truth = np.array([0.0, 0.1, 20.0, 0.6])
    t, tt, F, w = data(amap, truth)
    rng = np.random.default_rng(1)
    P = truth + np.stack([rng.normal(0, 2, 12), rng.normal(0, 0.05, 12), rng.normal(0, 2, 12),
                          rng.normal(0, 0.1, 12)], axis=1)
    _, g1, _, _ = chi2_grad(amap, WIN, tt, F, w, P)
    g2 = chi2_grad_explicit(amap, WIN, tt, F, w, P)
    scale = np.abs(g1).max(axis=1, keepdims=True)
    assert np.abs(g1 - g2).max() / scale.min() < 1e-8


def test_gradient_matches_central_differences():
    amap = smooth_map()
    truth = np.array([0.0, 0.1, 20.0, 0.6])
    t, tt, F, w = data(amap, truth, n=60)
    rng = np.random.default_rng(2)
    P = truth + np.stack([rng.normal(0, 2, 40), rng.normal(0, 0.05, 40), rng.normal(0, 2, 40),
                          rng.normal(0, 0.1, 40)], axis=1)
    _, g, _, _ = chi2_grad(amap, WIN, None, F, w, P, t=t, mode="exact64")
    fd, elig = fd_gradient(amap, WIN, t, F, w, P, rel=1e-7)
    assert elig.sum(axis=0).min() >= 5
    gmax = np.abs(g).max(axis=1, keepdims=True)
    tol = 1e-4 * np.maximum(np.abs(g), 1e-3 * gmax)
    assert (np.abs(fd - g) <= tol)[elig].all()


def test_lbfgs_decreases_and_converges_noise_free():
    amap = smooth_map()
    truth = np.array([0.0, 0.1, 20.0, 0.6])
    t, tt, F, w = data(amap, truth, noise=False)
    anchor = truth + np.array([0.4, 0.01, 0.8, 0.03])
    p, f, fs = refine_one(amap, WIN, tt, F, w, 0.0, anchor, LbfgsOptions(steps=80))
    assert all(b <= a for a, b in zip(fs, fs[1:]))
    assert f < 1e-3 * fs[0]
    assert np.abs(p - truth).max() < 1e-3


def test_lbfgs_batch_equals_single():
    amap = smooth_map()
    truth = np.array([0.0, 0.1, 20.0, 0.6])
    t, tt, F, w = data(amap, truth)
    anchors = truth + np.array([[0.4, 0.01, 0.8, 0.03], [-1.0, 0.02, -2.0, -0.05]])
    P, f, f0 = refine(amap, WIN, tt, F, w, 0.0, anchors, LbfgsOptions(steps=10))
    for i in range(2):
        p1, f1, _ = refine_one(amap, WIN, tt, F, w, 0.0, anchors[i], LbfgsOptions(steps=10))
        assert np.array_equal(p1, P[i]) and f1 == f[i]
        assert f[i] <= f0[i]


def test_fp64_gradient_matches_differences_on_a_ray_map():
    """The FP64 analytic gradient against central differences (step 1e-5 relative) on
    the tiny ray-shooting map (rough: about 10 rays per pixel), componentwise 1e-4."""
    import workloads as W
    from oracle.rays import rayshoot_mirror32_c
    from oracle.maps import map_scale
    c = W.config("tiny")
    counts, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=4)
    amap = (counts.astype(np.float32) * map_scale(c["rays"], c["window"])).astype(np.float32)
    ev = W.load_lightcurve("tiny")
    rng = np.random.default_rng(2)
    tr = ev["truth"]
    P = np.array([tr["t0"], tr["u0"], tr["tE"], tr["alpha"]]) + rng.normal(0, 1, (16, 4)) * [1.0, 0.02, 1.5, 0.05]
    _, g, _, _ = chi2_grad(amap, c["window"], None, ev["F"], ev["w"], P, ev["t_ref"], t=ev["t"],
                           mode="exact64")
    fd, elig = fd_gradient(amap, c["window"], ev["t"], ev["F"], ev["w"], P, ev["t_ref"], rel=1e-5)
    assert elig.sum() >= 8
    gmax = np.abs(fd).max(axis=1, keepdims=True)
    assert (np.abs(g - fd) <= 1e-4 * np.maximum(np.abs(fd), 1e-3 * gmax))[elig].all()
