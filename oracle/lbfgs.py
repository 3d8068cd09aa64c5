"""Batched L-BFGS refinement of grid candidates (test infrastructure only).

Refines (t0, u0, tE, alpha) of a candidate trajectory on its map by minimising the
profiled chi-square with the gradient of ``adjoint`` (mirror32 samples).  The paper
refines its seeds with MCMC (sec. 5); gradient refinement on the maps is the method
here, so the details below are choices of this refinement, fixed here and mirrored by the GPU.

Variables: the optimiser works on p in binary32, a scaled displacement from the
candidate's FP64 anchor (t0_i, u0_i, tE_i, a_i):
    t0 = t0_i + p0 tE_i,  u0 = u0_i + p1,  tE = tE_i exp(p2),  alpha = a_i + p3,
so d chi2/d p = (g_t0 tE_i, g_u0, g_tE tE, g_alpha).

One round = one chi-square/gradient evaluation at the trial point p_t, then:
  round 0: accept p = p_t (= 0) and take a new direction;
  later rounds, Armijo test f_t <= f + (c1 t) (g . d) (and f_t finite):
    pass: s = p_t - p, y = g_t - g (FP64); keep the pair when s.y > 1e-12 |s| |y|
          (history of at most m, oldest dropped); p, f, g = p_t, f_t, g_t; new direction;
    fail: n_ls += 1; stop the candidate when n_ls reaches max_ls, else t *= shrink and
          p_t = fl32(p + t d).
  New direction: two-loop recursion with H0 = gamma I, gamma = s.y / y.y of the newest
  pair (no pairs: gamma = 1e-2/|g|); d = -H g; if g.d >= 0 or non-finite, clear the
  history and use d = -(1e-2/|g|) g; t = 1, n_ls = 0, p_t = fl32(p + t d); a trial
  equal to p in every component stops the candidate.
Dot products are evaluated left to right over the 4 components without fused
multiply-add, so a binary32/FP64 implementation elsewhere can reproduce the state
machine exactly given the same chi-square and gradients.
"""
from __future__ import annotations

import math

import numpy as np

from .adjoint import chi2_grad

__all__ = ["LbfgsOptions", "natural_params", "two_loop_direction", "store_pair", "minimize",
           "refine_one", "refine"]


class LbfgsOptions:
    def __init__(self, steps=50, history=8, max_ls=10, c1=1e-4, shrink=0.5):
        self.steps = steps
        self.history = history
        self.max_ls = max_ls
        self.c1 = c1
        self.shrink = shrink


def _dot(a, b):
    return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3]


def natural_params(anchor, p):
    t0, u0, tE, al = (float(v) for v in anchor)
    p = [float(np.float32(v)) for v in p]
    return np.array([t0 + p[0] * tE, u0 + p[1], tE * math.exp(p[2]), al + p[3]])


def _eval(amap, window, tt, F, w, t_ref, anchor, p):
    th = natural_params(anchor, p)
    chi2, g, _, _ = chi2_grad(amap, window, tt, F, w, th[None, :], t_ref)
    g = g[0]
    gp = [g[0] * float(anchor[2]), g[1], g[2] * th[2], g[3]]
    return float(chi2[0]), gp


def two_loop_direction(S, Y, R, g):
    """d = -H g by the two-loop recursion over the stored pairs (oldest first), with
    H0 = gamma I, gamma = s.y / y.y of the newest pair (no pairs: 1e-2/|g|)."""
    q = list(g)
    alph = []
    for i in range(len(S) - 1, -1, -1):
        a = R[i] * _dot(S[i], q)
        alph.append(a)
        q = [q[k] - a * Y[i][k] for k in range(4)]
    alph.reverse()
    gn = math.sqrt(_dot(g, g))
    if S:
        gamma = _dot(S[-1], Y[-1]) / _dot(Y[-1], Y[-1])
    else:
        gamma = 1e-2 / gn if gn > 0 else 0.0
    r = [gamma * q[k] for k in range(4)]
    for i in range(len(S)):
        b = R[i] * _dot(Y[i], r)
        r = [r[k] + S[i][k] * (alph[i] - b) for k in range(4)]
    return [-r[k] for k in range(4)]


def store_pair(S, Y, R, s, y, m):
    """Append the curvature pair (s, y) when s.y > 1e-12 |s| |y|, dropping the oldest
    pair beyond m; returns whether the pair was kept."""
    sy = _dot(s, y)
    if not sy > 1e-12 * math.sqrt(_dot(s, s)) * math.sqrt(_dot(y, y)):
        return False
    S.append(list(s))
    Y.append(list(y))
    R.append(1.0 / sy)
    while len(S) > m:
        S.pop(0)
        Y.pop(0)
        R.pop(0)
    return True


def minimize(evaluate, opt: LbfgsOptions, trace=None):
    """Run the state machine above on evaluate(p) -> (f, grad) (p: 4 binary32 values,
    grad: 4 floats); returns (p, f, history of accepted f).  When trace is a list, each
    new direction appends a dict with the accepted point p, its f and g, the direction
    d and the number of stored pairs."""
    S, Y, R = [], [], []
    p = [np.float32(0.0)] * 4
    pt = [np.float32(0.0)] * 4
    f = g = d = None
    t = 1.0
    nls = 0
    active = True
    fs = []

    def new_direction():
        nonlocal d, t, nls, pt, active, S, Y, R
        d = two_loop_direction(S, Y, R, g)
        gd = _dot(g, d)
        if not (gd < 0.0) or not all(math.isfinite(v) for v in d):
            S, Y, R = [], [], []
            gn = math.sqrt(_dot(g, g))
            gamma = 1e-2 / gn if gn > 0 else 0.0
            d = [-(gamma * g[k]) for k in range(4)]
        if trace is not None:
            trace.append({"p": [float(v) for v in p], "f": f, "g": list(g), "d": list(d),
                          "pairs": len(S)})
        t = 1.0
        nls = 0
        pt = [np.float32(float(p[k]) + t * d[k]) for k in range(4)]
        if all(pt[k] == p[k] for k in range(4)):
            active = False

    for rnd in range(opt.steps + 1):
        if not active:
            break
        ft, gt = evaluate(pt)
        if rnd == 0:
            p, f, g = list(pt), ft, gt
            fs.append(f)
            new_direction()
            continue
        gd = _dot(g, d)
        if math.isfinite(ft) and ft <= f + (opt.c1 * t) * gd:
            s = [float(pt[k]) - float(p[k]) for k in range(4)]
            y = [gt[k] - g[k] for k in range(4)]
            store_pair(S, Y, R, s, y, opt.history)
            p, f, g = list(pt), ft, gt
            fs.append(f)
            new_direction()
        else:
            nls += 1
            if nls >= opt.max_ls:
                active = False
            else:
                t *= opt.shrink
                pt = [np.float32(float(p[k]) + t * d[k]) for k in range(4)]
    return p, f, fs


def refine_one(amap, window, tt, F, w, t_ref, anchor, opt: LbfgsOptions, trace=None):
    """Refine one candidate; returns (natural params [4], chi2, history of f)."""
    p, f, fs = minimize(lambda pt: _eval(amap, window, tt, F, w, t_ref, anchor, pt), opt, trace)
    return natural_params(anchor, p), f, fs


def refine(amap, window, tt, F, w, t_ref, anchors, opt: LbfgsOptions = None):
    """Refine each row of anchors [n, 4]; returns (params [n, 4], chi2 [n], f0 [n])."""
    opt = opt or LbfgsOptions()
    anchors = np.asarray(anchors, dtype=np.float64).reshape(-1, 4)
    out = np.zeros_like(anchors)
    chi = np.zeros(len(anchors))
    f0 = np.zeros(len(anchors))
    for i, a in enumerate(anchors):
        out[i], chi[i], fs = refine_one(amap, window, tt, F, w, t_ref, a, opt)
        f0[i] = fs[0]
    return out, chi, f0
