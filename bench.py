#!/usr/bin/env python3
"""Benchmark of the MORSE map-build + trajectory-search hot path on one MI355X.

One step = the whole path over the batched-events workload, the largest configuration:
  * the 64-map (s, q) bank built twice from rays: at 1024^2 from 16384^2 rays each (the
    search maps, point source) and at 2048^2 from 32768^2 rays each (the refinement
    maps): ray shooting, binning and normalisation, 8.6e10 rays;
  * the batched (persistent, graph-replayed) chi-square search of 256 ragged events
    (200..20000 points, 903,548 in all) x 64 maps x 32768 trajectories per event,
    1.9e12 light-curve point-evaluations, with the top 4096 (chi2, map, trajectory) of
    every event;
  * 50 L-BFGS rounds with the chi-square adjoint of the top 4096 candidates of the first
    64 events (262,144 candidates) on their 2048^2 maps.

value = search point-evaluations per second of the whole step (map builds and the
refinement charged to the same clock), steps one after another in the library's
production schedule (graph-replayed search, two-stream refinement, no per-kernel
timing).  A separate pass times each kernel family with HIP events around its launches
for the roofline.  Also reported: rays/s, the plain (one launch per event and map)
search of the same problem, the adjoint rate, the (s, q)-grid workload (384 maps) and
the large single-map workload with the finite-source stack, the caustic-line filter and
the line simplex, and the CPU oracle on this host (single thread and all cores).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic lane-operations per unit (one FP32/FP64 add, mul, compare, floor,
# convert, divide, square root or fused multiply-add = 1), split by the unit that
# executes them, (binary32 and integer, FP64):
#   ray, shot in mirror pairs (one lens-equation solve for a ray and its image across
#        the lens axis): per pair lattice point 2, d 2, r 4, two divisions 2,
#        zeta_x 4, zeta_y 4, scaled offsets 4, floors 2, bin compares/selects 4,
#        mirror row 1, and per ray index 2, count 1: 35 per pair    = (17.5, 0)
#   point-evaluation: tau 2, zeta 4, grid coordinate 6, on-map test 4,
#        floor/fraction 4, cell index 3, bilinear 9 (binary32) + FP64 sums 5 = (32, 5)
#   adjoint point-evaluation: sample 32 (binary32) + fit sums 5, dA/dzeta 5, tau and
#        alpha directions 5, five directions x (w D and three sums) 20 (FP64) = (32, 35)
OPS_PER_RAY = (17.5, 0)
OPS_PER_POINT_EVAL = (32, 5)
OPS_PER_ADJOINT_EVAL = (32, 35)
# Vector peaks of one MI355X in lane-operations per second (an FMA counts once, so
# these are half the published 157.3 TFLOP/s binary32 and 78.6 TFLOP/s FP64):
# 256 CUs x 2.4 GHz x 128 binary32 lanes / 64 FP64 lanes per clock.
PEAK_F32 = 256 * 2.4e9 * 128
PEAK_F64 = 256 * 2.4e9 * 64
HBM_PEAK_GBS = 8000.0


def peak_for(ops):
    """Peak lane-op rate of a unit of work with (binary32, FP64) operation counts."""
    n32, n64 = ops
    return (n32 + n64) / (n32 / PEAK_F32 + n64 / PEAK_F64)


# HBM-side traffic per launch (bytes) of a kernel on a workload, from two rocprofv3
# --pmc runs of this bench (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled
# by what the same counter reads for a 1 GiB device-to-device copy (FETCH_SIZE at most
# 524308 KiB: factor 1.99992; WRITE_SIZE 1048576 KiB: factor 1.0).  Keyed by the kernel, a
# hash of the sources it is built from and the workload; a changed kernel reports null
# until it is measured again.  Batched-events workload: the search's full launch
# (FETCH 9.41794e+08 KiB, WRITE 2.32661e+07 KiB), the gradient's full 262144-candidate
# launch (1.00305e+07, 14766.7 KiB) and the mean over the two map sizes of the ray kernel
# (FETCH 241.05 and 238.9 KiB, WRITE 68854.7 and 17281.9 KiB).
TRAFFIC = {
    ("k_search_batched", "95093939f55768c2", "batched"): 1.952545e+12,
    ("k_chi2_grad", "98c959850a2a8b8a", "batched"): 2.055676e+10,
    ("k_rayshoot", "eae3ebd5e214d8e9", "batched"): 4.459335e+07,
}
STACK_GAMMA = 0.53        # limb-darkening coefficient of the finite-source stack
STACK_FFT_MIN_TAPS = 256  # the library's default split between direct sums and transforms
KERNEL_SOURCES = {"k_rayshoot": ("maps.hip", "internal.h"),
                  "k_search_batched": ("search.hip", "internal.h"),
                  "k_chi2_grad": ("refine.hip", "internal.h")}
CPU_WORKERS = 16          # the host-core share of one GPU
TU1_SHAPE = 1             # the library's batched-search shape (8, 4, 16, TU = 1)


def kernel_sha(kernel):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1511_01157_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel-steps", type=int, default=2,
                    help="steps of the separate per-kernel timing pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-sqgrid", action="store_true", help="skip the (s, q)-grid workload")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large single-map workload (and its stack / line rows)")
    ap.add_argument("--large-steps", type=int, default=5)
    # profiling aids: a plain device copy of known size (the reference for scaling
    # the FETCH_SIZE / WRITE_SIZE counters), and text summaries of rocprofv3 output
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run 5 device-to-device copies of this many bytes")
    ap.add_argument("--summarize-trace", metavar="RESULTS_DB",
                    help="print a per-kernel table of a rocprofv3 --kernel-trace database")
    ap.add_argument("--summarize-pmc", metavar="COUNTER_CSV", nargs="+",
                    help="print per-kernel means per dispatch of rocprofv3 --pmc CSV files")
    return ap.parse_args()


def short_name(name):
    import re
    m = re.search(r"(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name.split("(")[0][-40:]


def summarize_trace(path):
    import sqlite3
    cur = sqlite3.connect(path).cursor()
    # the gradient kernel is listed per grid size: a refinement of many candidates runs
    # two half-size chains side by side, a timed or small one a single full-size chain
    rows = cur.execute(
        "select name, case when name like '%k_chi2_grad%' then grid_x else 0 end, count(*), "
        "sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(sgpr_count), max(lds_size) from kernels group by 1, 2 "
        "order by sum(duration) desc").fetchall()
    tot = sum(r[3] for r in rows)
    print("| kernel | calls | total ms | avg us | min us | max us | % | VGPR | SGPR | LDS B |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for n, g, c, t, a, mn, mx, v, sg, lds in rows:
        label = short_name(n) + (f" (grid_x {g})" if g else "")
        print(f"| {label} | {c} | {t / 1e6:.3f} | {a / 1e3:.2f} | {mn / 1e3:.2f} | "
              f"{mx / 1e3:.2f} | {100 * t / tot:.2f} | {v} | {sg} | {lds} |")


def summarize_pmc(paths):
    import csv
    from collections import defaultdict
    acc = defaultdict(list)
    for path in paths:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                acc[(short_name(row["Kernel_Name"]), row["Counter_Name"])].append(
                    float(row["Counter_Value"]))
    print("| kernel | counter | dispatches | mean per dispatch | min | max |")
    print("|---|---|---|---|---|---|")
    for (k, cn), v in sorted(acc.items()):
        print(f"| {k} | {cn} | {len(v)} | {sum(v) / len(v):.6g} | {min(v):.6g} | {max(v):.6g} |")
    # the same kernel also runs on sub-problems (the autotuner's, a warm-up's); the
    # dispatches within a factor 4 of the largest are the full-size launches
    print()
    print("Full-size dispatches (counter value at least a quarter of the kernel's largest):")
    print()
    print("| kernel | counter | dispatches | mean per dispatch | min | max |")
    print("|---|---|---|---|---|---|")
    for (k, cn), v in sorted(acc.items()):
        big = [x for x in v if x >= 0.25 * max(v)]
        if len(big) < len(v):
            print(f"| {k} | {cn} | {len(big)} | {sum(big) / len(big):.6g} | {min(big):.6g} | "
                  f"{max(big):.6g} |")


def copy_kernel(nbytes):
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes x 5", flush=True)


def roofline(kernel, ops, units, total_ms, launches, workload, upper=False):
    """Roofline record of one kernel family: algorithmic lane-operations of all its
    timed launches over their summed launch times."""
    peak = peak_for(ops) / 1e12
    ms = total_ms / max(launches, 1)
    achieved = sum(ops) * units / (total_ms * 1e-3) / 1e12
    traffic = TRAFFIC.get((kernel, kernel_sha(kernel), workload))
    return {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "traffic_gbs": traffic / (ms * 1e-3) / 1e9 if traffic else None,
            "traffic_frac_of_hbm": traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
            "launch_ms": ms, "launches": launches,
            "ops_per_launch": sum(ops) * units / max(launches, 1),
            "ops_are_upper_bound": upper, "ops_per_unit_f32_f64": list(ops)}


OP_NOTE = ("achieved and peak in tera lane-operations/s (one FP32/FP64 add, mul, compare, "
           "floor, cvt, div, sqrt or FMA per lane = 1); peak = the kernel's binary32/FP64 op "
           "mix at 256 CU x 2.4 GHz x 128 binary32 or 64 FP64 lanes per clock (half the "
           "published 157.3/78.6 TFLOP/s, which count an FMA twice); launch times from HIP "
           "events around each launch on the library's stream, in a pass apart from the "
           "timed steps; traffic from rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, "
           "calibrated on a device copy")


# ----------------------------------------------------------------------------------
# CPU baseline: the oracle as it stands on this host's cores, on a bounded sample of
# one step of the batched-events workload, single thread and CPU_WORKERS processes,
# each figure the median of three runs.  It runs before anything touches the GPU (the
# worker processes are forked from this one).
_CB = {}


def _cb_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _cb_search(task):
    """Oracle search of one event's first n trajectories on the sample map; returns
    (seconds, point-evaluations, the best trajectory)."""
    from oracle.search import search_mirror32
    e, n = task
    ev = _CB["events"][e]
    P = _CB["P"][e][:n]
    t = time.perf_counter()
    chi2 = search_mirror32(_CB["map1"], _CB["win1"], ev["tt"], ev["F"], ev["w"], P, ev["t_ref"])[0]
    return time.perf_counter() - t, n * len(ev["tt"]), P[int(chi2.argmin())]


CB_REFINE_ROUNDS = 10  # L-BFGS rounds timed per candidate (one evaluation each)


def _cb_refine(task):
    """Oracle L-BFGS of one candidate on the 2048^2 sample map, CB_REFINE_ROUNDS rounds
    after the first evaluation; returns (seconds, candidate-round-points)."""
    import numpy as np
    from oracle.lbfgs import LbfgsOptions, refine
    e, anchor = task
    ev = _CB["events"][e]
    t = time.perf_counter()
    with np.errstate(all="ignore"):  # trial points far out give non-finite chi2, rejected
        refine(_CB["map2"], _CB["win2"], ev["tt"], ev["F"], ev["w"], ev["t_ref"], anchor[None, :],
               LbfgsOptions(steps=CB_REFINE_ROUNDS))
    return time.perf_counter() - t, (CB_REFINE_ROUNDS + 1) * len(ev["tt"])


def _cb_norm(task):
    """Oracle normalisation (point source: scale only) of the 2048^2 sample counts."""
    from oracle.maps import normalize_convolve_mirror32
    t = time.perf_counter()
    normalize_convolve_mirror32(_CB["counts2"], _CB["scale2"], _CB["w0"])
    return time.perf_counter() - t, _CB["counts2"].size


def _median_rate(fn, reps=3):
    rates = sorted(fn() for _ in range(reps))
    return rates[len(rates) // 2]


def cpu_baseline_batched(units):
    """units: the step's rays, map pixels, search point-evaluations and refinement
    candidate-round-points (candidates x evaluations x points).  Returns the
    cpu_baseline record."""
    import multiprocessing as mp
    import platform

    import numpy as np
    import workloads as W
    from oracle.maps import disk_pixel_weights, map_scale
    from oracle.rays import rayshoot_mirror32_c

    nw = max(1, min(CPU_WORKERS, os.cpu_count() or 1))
    cb, cr = W.config("batched"), W.config("refine")
    bank = W.map_bank("batched")
    mi = 27  # a mid-bank (s, q) with a resonant-size caustic
    s, q = bank[mi]
    progress(f"cpu baseline: oracle maps s={s:.3g} q={q:.3g} at 1024^2 and 2048^2")
    c1, _ = rayshoot_mirror32_c(s, q, cb["rays"], cb["window"], nthreads=nw)
    c2, _ = rayshoot_mirror32_c(s, q, cr["rays"], cr["window"], nthreads=nw)
    w0 = disk_pixel_weights(0.0, 1, 1)
    from oracle.maps import normalize_convolve_mirror32
    # events of the refinement set (the first 64) nearest the median length
    lens = np.array([t["npts"] for t in W.truths("refine")])
    pick = [int(e) for e in np.argsort(np.abs(lens - np.median(lens)))[:nw]]
    _CB.update(map1=normalize_convolve_mirror32(c1, map_scale(cb["rays"], cb["window"]), w0),
               map2=normalize_convolve_mirror32(c2, map_scale(cr["rays"], cr["window"]), w0),
               win1=cb["window"], win2=cr["window"], counts2=c2, w0=w0,
               scale2=map_scale(cr["rays"], cr["window"]),
               events={e: W.load_lightcurve("batched", e) for e in pick},
               P={e: W.random_trajectories("batched", e) for e in pick})
    _cb_init()
    n_tr = 512
    pool = mp.get_context("fork").Pool(nw, initializer=_cb_init)
    try:
        def pool_rate(fn, tasks):
            t = time.perf_counter()
            res = pool.map(fn, tasks)
            return sum(r[1] for r in res) / (time.perf_counter() - t), res

        progress("cpu baseline: rays")
        ny = cb["rays"][5]

        def rays_rate(threads, rows):
            j0 = ny // 2 - rows // 2
            t = time.perf_counter()
            rayshoot_mirror32_c(s, q, cb["rays"], cb["window"], rows=(j0, j0 + rows), nthreads=threads)
            return rows * cb["rays"][4] / (time.perf_counter() - t)
        r_rays = (_median_rate(lambda: rays_rate(1, 256)), _median_rate(lambda: rays_rate(nw, 256 * nw)))
        progress("cpu baseline: normalisation")
        r_norm = (_median_rate(lambda: (lambda r: r[1] / r[0])(_cb_norm(None))),
                  _median_rate(lambda: pool_rate(_cb_norm, [None] * nw)[0]))
        progress("cpu baseline: search")
        r_s1 = _median_rate(lambda: (lambda r: r[1] / r[0])(_cb_search((pick[0], n_tr))))
        runs = [pool_rate(_cb_search, [(e, n_tr) for e in pick]) for _ in range(3)]
        r_sa = sorted(r for r, _ in runs)[1]
        seeds = [(e, r[2]) for e, r in zip(pick, runs[0][1])]  # the oracle's own best per event
        progress("cpu baseline: refinement")
        r_c1 = _median_rate(lambda: (lambda r: r[1] / r[0])(_cb_refine(seeds[0])))
        r_ca = _median_rate(lambda: pool_rate(_cb_refine, seeds)[0])
    finally:
        pool.terminate()
        pool.join()
    out = {}
    for j, (label, cores) in enumerate((("single_thread", 1), ("all_cores", nw))):
        rr, rn, rs, rc = r_rays[j], r_norm[j], (r_s1, r_sa)[j], (r_c1, r_ca)[j]
        t = {"rays": units["rays"] / rr, "normalise": units["pixels"] / rn,
             "search": units["evals"] / rs, "refine": units["cand_round_points"] / rc}
        out[label] = {"value": units["evals"] / sum(t.values()), "cores": cores,
                      "step_s": sum(t.values()), "leg_s": t,
                      "rates": {"rays_per_s": rr, "pixels_per_s": rn, "point_evals_per_s": rs,
                                "candidate_round_points_per_s": rc}}
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except Exception:
        model = platform.processor()
    return {
        "value": out["all_cores"]["value"], "unit": "point-evals/s", "cores": nw, "kind": "oracle",
        "sample": (f"one batched-events step extrapolated from timed samples, median of 3 each, "
                   f"on map {mi} of the bank (s={s:.3g}, q={q:.3g}): C binary32 ray mirror on 256 "
                   f"central lattice rows per thread; normalisation of the 2048^2 counts once per "
                   f"process; numpy binary32 search of {n_tr} trajectories of one event per "
                   f"process ({len(pick)} events of median length); numpy L-BFGS (FP64 adjoint) of "
                   f"each event's best sampled trajectory on the 2048^2 map, {CB_REFINE_ROUNDS} "
                   f"rounds timed and scaled per round to the step's 51 evaluations; "
                   f"all-core figures from {nw} forked processes (wall clock), single-thread "
                   f"from one; each leg scaled by the step's own units"),
        "single_thread": out["single_thread"], "all_cores": out["all_cores"],
        "host": {"cpu": model, "nproc": os.cpu_count()},
    }


# ----------------------------------------------------------------------------------
# GPU legs
def events_timer(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def leg_batched(args, M, W, torch, np, dev):
    """The headline step on the batched-events workload (module docstring)."""
    cb, cr = W.config("batched"), W.config("refine")
    bank = W.map_bank("batched")
    n_ev, n_r, k = cb["n_events"], cr["n_events"], cr["top_k"]
    evs = [W.load_lightcurve("batched", e) for e in range(n_ev)]
    P = np.stack([W.random_trajectories("batched", e) for e in range(n_ev)])
    n_pts = np.array([len(e["tt"]) for e in evs])
    n_traj = P.shape[1]
    stream = torch.cuda.Stream(device=dev)
    ctx = M.Context.bound(stream)
    (w1, r1), (w2, r2) = (cb["window"], cb["rays"]), (cr["window"], cr["rays"])
    units = {"rays": len(bank) * (r1[4] * r1[5] + r2[4] * r2[5]),
             "pixels": len(bank) * (w1[4] * w1[5] + w2[4] * w2[5]),
             "evals": int(n_pts.sum()) * len(bank) * n_traj,
             "cand_points": k * int(n_pts[:n_r].sum())}
    with torch.cuda.stream(stream):
        lcs = M.LightCurveBatch.from_events(evs, dev)
        Pd = torch.from_numpy(P).to(dev)
        trajs = M.list_trajectories(Pd, shared=False)
        trajs_r = M.list_trajectories(Pd[:n_r], shared=False)
        bank1 = torch.empty((len(bank), w1[5], w1[4]), dtype=torch.float32, device=dev)
        bank2 = torch.empty((len(bank), w2[5], w2[4]), dtype=torch.float32, device=dev)
        cnt1 = torch.empty((w1[5], w1[4]), dtype=torch.int32, device=dev)
        cnt2 = torch.empty((w2[5], w2[4]), dtype=torch.int32, device=dev)
        views1 = [(bank1[i], w1) for i in range(len(bank))]
        views2 = [(bank2[i], w2) for i in range(len(bank))]
        sbuf = {}
        cand = (torch.empty((n_r * k, 4), dtype=torch.float64, device=dev),
                torch.empty(n_r * k, dtype=torch.int32, device=dev),
                torch.empty(n_r * k, dtype=torch.int32, device=dev))
        rbuf = (torch.empty(n_r * k, dtype=torch.float64, device=dev),
                torch.empty(n_r * k, dtype=torch.float64, device=dev))

        def build_bank(cfg, maps, cnt):
            for i, (s, q) in enumerate(bank):
                M.rayshoot(s, q, cfg["rays"], cfg["window"], cnt, ctx=ctx)
                M.normalize_convolve(cnt, cfg["rays"], cfg["window"], cfg["rho"], out=maps[i], ctx=ctx)

        def step(ev=None):
            mark = (lambda j: ev[j].record(stream)) if ev else (lambda j: None)
            mark(0)
            build_bank(cb, bank1, cnt1)
            build_bank(cr, bank2, cnt2)
            mark(1)
            r = M.search(views1, lcs, trajs, "batched", chi2=False, top_k=k, out=sbuf, ctx=ctx)
            sbuf.update(r)
            mark(2)
            Pc, e_idx, m_idx = M.candidates_from_topk(trajs_r, r["topk_idx"][:n_r], len(bank),
                                                      out=cand, ctx=ctx)
            out, chi2, chi2_0 = M.refine(views2, lcs, Pc, e_idx, m_idx, steps=cr["steps"],
                                         inplace=True, chi2_out=rbuf, ctx=ctx)
            mark(3)
            return chi2, chi2_0

        progress("batched: bank build + autotune")
        build_bank(cb, bank1, cnt1)
        import tempfile
        tune_path = os.path.join(tempfile.mkdtemp(prefix="morse_bench_"), "tune.json")
        tuned = M.autotune(views1, lcs, trajs, cache_path=tune_path, ctx=ctx)
        progress(f"batched: warm-up x{max(1, args.warmup)} (autotuned shape {tuned})")
        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        progress(f"batched: {args.steps} timed steps")
        ev = [events_timer(torch, 4) for _ in range(args.steps)]
        t0, t1 = events_timer(torch, 2)
        torch.cuda.synchronize()
        t0.record(stream)
        wall0 = time.perf_counter()
        for i in range(args.steps):
            res = step(ev[i])
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms_step = t0.elapsed_time(t1) / args.steps
        stage = np.mean([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in ev], axis=0)
        chi2, chi2_0 = res
        improved = float((chi2 <= chi2_0).float().mean())
        strictly = float((chi2 < chi2_0).float().mean())

        # kernel times: a separate pass with HIP events around every launch of each
        # family (the refinement then runs as one chain of launches)
        ks = max(1, args.kernel_steps)
        progress(f"batched: kernel timing pass x{ks}")
        fams = {"k_rayshoot": M.KERNEL_RAYSHOOT, "k_search_batched": M.KERNEL_SEARCH,
                "k_chi2_grad": M.KERNEL_GRADIENT}
        ctx.set_timing(list(fams.values()))
        for f in fams.values():
            ctx.kernel_time(f, reset=True)
        for _ in range(ks):
            step()
        torch.cuda.synchronize()
        ktime = {n: ctx.kernel_time(f, reset=True) for n, f in fams.items()}
        ctx.set_timing([])

        plain_ms = tu1_ms = same_tu1 = None
        if not args.no_plain:
            progress("batched: plain search (one launch per event and map)")
            pbuf = {}
            e0, e1 = events_timer(torch, 2)
            torch.cuda.synchronize()
            e0.record(stream)
            pr = M.search(views1, lcs, trajs, "plain", chi2=False, top_k=k, out=pbuf, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            plain_ms = e0.elapsed_time(e1)
            same_topk = bool(torch.equal(pr["topk_idx"], sbuf["topk_idx"]) and
                             torch.equal(pr["topk_chi2"], sbuf["topk_chi2"]))
            # the batched kernel at a TU = 1 shape of its table, which separates the one
            # persistent launch from scoring several trajectories per wavefront
            progress("batched: persistent search at TU = 1")
            with open(tune_path) as f:
                classes = json.load(f)
            with open(tune_path + ".tu1", "w") as f:
                json.dump({cl: TU1_SHAPE for cl in classes}, f)
            M.autotune_load(tune_path + ".tu1", ctx=ctx)
            b1 = {}
            b1 = M.search(views1, lcs, trajs, "batched", chi2=False, top_k=k, out=b1, ctx=ctx)
            torch.cuda.synchronize()
            e0.record(stream)
            b1 = M.search(views1, lcs, trajs, "batched", chi2=False, top_k=k, out=b1, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            tu1_ms = e0.elapsed_time(e1)
            same_tu1 = bool(torch.equal(b1["topk_idx"], sbuf["topk_idx"]) and
                            torch.equal(b1["topk_chi2"], sbuf["topk_chi2"]))
            M.autotune_load(tune_path, ctx=ctx)  # the tuned shape again

    build_ms, search_ms, refine_ms = stage
    rounds = cr["steps"] + 1
    kr = {
        "k_rayshoot": roofline("k_rayshoot", OPS_PER_RAY, ks * units["rays"], *ktime["k_rayshoot"],
                               "batched"),
        "k_search_batched": roofline("k_search_batched", OPS_PER_POINT_EVAL, ks * units["evals"],
                                     *ktime["k_search_batched"], "batched"),
        "k_chi2_grad": roofline("k_chi2_grad", OPS_PER_ADJOINT_EVAL,
                                ks * rounds * units["cand_points"], *ktime["k_chi2_grad"],
                                "batched", upper=True),
    }
    per_step = {n: t / ks for n, (t, _) in ktime.items()}
    dom = max(per_step, key=per_step.get)
    rec = {
        "ms_per_step": ms_step, "wall_s_timed": wall,
        "value": units["evals"] / (ms_step * 1e-3),
        "stages_ms": {"map_banks": build_ms, "search_batched": search_ms,
                      "candidates_refine": refine_ms},
        "rays_per_s": units["rays"] / (build_ms * 1e-3),
        "search_point_evals_per_s": {
            "batched": units["evals"] / (search_ms * 1e-3),
            "plain": units["evals"] / (plain_ms * 1e-3) if plain_ms else None,
            "batched_tu1": units["evals"] / (tu1_ms * 1e-3) if tu1_ms else None,
            "batched_tu1_shape": (f"entry {TU1_SHAPE} of the library's shape table: 8 trajectories "
                                  "per item, 4 waves per workgroup, 16 workgroups per CU, TU = 1; "
                                  f"top-k equal to the tuned run: {same_tu1}"),
            "batched_shape": {"autotuned_index": tuned, "note": "trajectories per item, waves "
                              "per workgroup, workgroups per CU and TU of the library's shape "
                              "table entry; one persistent launch over (event, map, trajectory "
                              "block) items, graph-replayed"},
            "plain_shape": "one launch per (event, map): one wavefront per trajectory (TU = 1), "
                           "4 wavefronts per workgroup",
            "plain_topk_equal": same_topk if plain_ms else None},
        "adjoint_point_evals_per_s_upper": rounds * units["cand_points"] / (refine_ms * 1e-3),
        "refine_chi2_not_raised": improved, "refine_chi2_lowered": strictly,
        "kernel_ms_per_step": per_step, "kernels": kr, "dominant": dom,
        "units": units,
        "config": {"workload": ("batched events: 256 ragged events (lognormal lengths, median "
                                "2000, 200-20000 points, 903548 in all) x 64-map (s, q) bank at "
                                "1024^2 from 16384^2 rays each, point source, x 32768 random "
                                "trajectories per event per map, top-4096 per event; then 50 "
                                "L-BFGS rounds of the top-4096 of the first 64 events (262144 "
                                "candidates) on the bank rebuilt at 2048^2 from 32768^2 rays"),
                   "n_events": n_ev, "n_maps": len(bank), "n_traj_per_event": n_traj,
                   "n_points": int(n_pts.sum()), "maps": [[w1[5], w1[4]], [w2[5], w2[4]]],
                   "rays_per_map": [r1[4] * r1[5], r2[4] * r2[5]], "top_k": k,
                   "refine_events": n_r, "refine_rounds": cr["steps"],
                   "parallelism": "single GPU", "autotuned_search_shape": tuned},
    }
    del bank1, bank2, sbuf, cand, rbuf
    torch.cuda.empty_cache()
    return rec


def leg_sqgrid(args, M, W, torch, np, dev):
    """(s, q) grid: 384 maps of 16384^2 rays at 1024^2 (rho = 1e-3, the identity), one
    3000-point light curve, 1e5 random trajectories shared by all maps, best per map."""
    c = W.config("sqgrid")
    bank = W.map_bank("sqgrid")
    ev = W.load_lightcurve("sqgrid")
    P = W.random_trajectories("sqgrid")
    win, rays = c["window"], c["rays"]
    stream = torch.cuda.Stream(device=dev)
    ctx = M.Context.bound(stream)
    n_rays = len(bank) * rays[4] * rays[5]
    evals = len(bank) * len(P) * len(ev["tt"])
    with torch.cuda.stream(stream):
        maps = torch.empty((len(bank), win[5], win[4]), dtype=torch.float32, device=dev)
        cnt = torch.empty((win[5], win[4]), dtype=torch.int32, device=dev)
        views = [(maps[i], win) for i in range(len(bank))]
        lcs = M.LightCurveBatch.from_events([ev], dev)
        trajs = M.list_trajectories(torch.from_numpy(P).to(dev))
        out = {}

        def step(e=None):
            mark = (lambda j: e[j].record(stream)) if e else (lambda j: None)
            mark(0)
            for i, (s, q) in enumerate(bank):
                M.rayshoot(s, q, rays, win, cnt, ctx=ctx)
                M.normalize_convolve(cnt, rays, win, c["rho"], out=maps[i], ctx=ctx)
            mark(1)
            r = M.search(views, lcs, trajs, "batched", chi2=False, best=True, out=out, ctx=ctx)
            out.update(r)
            mark(2)
            return r

        progress("sqgrid: 384 maps, autotune, warm-up")
        step()
        tuned = M.autotune(views, lcs, trajs, ctx=ctx)
        step()
        n = 3
        ev_ = [events_timer(torch, 3) for _ in range(n)]
        torch.cuda.synchronize()
        for i in range(n):
            r = step(ev_[i])
        torch.cuda.synchronize()
        st = np.mean([[e[j].elapsed_time(e[j + 1]) for j in range(2)] for e in ev_], axis=0)
        plain_ms = tu1_ms = same_tu1 = None
        if not args.no_plain:
            progress("sqgrid: plain search")
            e0, e1 = events_timer(torch, 2)
            e0.record(stream)
            M.search(views, lcs, trajs, "plain", chi2=False, best=True, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            plain_ms = e0.elapsed_time(e1)
        best = r["best_chi2"][0].cpu().numpy()
    mb = int(np.argmin(best))
    rec = {"workload": "(s, q) grid: 24 s x 16 q = 384 maps at 1024^2 from 16384^2 rays each, "
                       "rho = 1e-3 (the identity at this pixel size), one 3000-point light "
                       "curve, 1e5 random trajectories shared by all maps, best per map",
           "ms_per_step": float(sum(st)), "stages_ms": {"maps": st[0], "search_batched": st[1]},
           "rays_per_s": n_rays / (st[0] * 1e-3),
           "search_point_evals_per_s": {"batched": evals / (st[1] * 1e-3),
                                        "plain": evals / (plain_ms * 1e-3) if plain_ms else None},
           "autotuned_search_shape": tuned, "rays": n_rays, "point_evals": evals,
           "best_map": {"index": mb, "s": float(bank[mb][0]), "q": float(bank[mb][1]),
                        "chi2": float(best[mb])},
           "truth": {"s": c["s"], "q": c["q"]},
           "best_chi2_quantiles": [float(v) for v in np.quantile(best, [0.0, 0.5, 1.0])]}
    del maps
    torch.cuda.empty_cache()
    return rec


# Algorithmic work of the rows measured beside the large workload's step:
# one line-filter sample = tau 2, position 2, zeta 4, grid coordinates 4, on-map tests
# 4, floor/fraction 4, cell index 3, bilinear blend 9, max 1 (binary32/integer); one
# point of a simplex chi-square evaluation = the search's sample (32) + b, w b and the
# three FP64 sums (6); one lens-equation sample of the image-centred integration (FP64)
# = radius 2, position 2, offsets from the lenses 2, y^2 1, two squared distances 4,
# two divisions 2, the image position 10, squared distance to the source 3, the limb
# test 2.
OPS_PER_FILTER_SAMPLE = (33, 0)
OPS_PER_SIMPLEX_POINT = (32, 6)
OPS_PER_FS_SAMPLE = (0, 28)
FS_THETA, FS_R, FS_SHRINK = 512, 512, 2   # the library's image-centred grid and passes


def fft_passes(n):
    p, ns = 0, 1
    while ns < n:
        ns *= 16 if n // ns >= 16 else n // ns
        p += 1
    return p


def stack_bytes(mx, my, nx, ny, n_fft, n_direct):
    """Algorithmic HBM bytes of one stack call: the counts' forward transform (map rows,
    half spectrum), one inverse per pair of FFT radii, and the direct radii (4 B of
    counts read and 4 B of map written per pixel each)."""
    h = nx // 2 + 1
    P = fft_passes(ny)
    fwd = mx * my * 4 + my * h * 16 + (my * h * 16 + ny * h * 16) + (P - 1) * 2 * ny * h * 16
    inv = (ny * h * 16 + 2 * ny * nx * 16) + (P - 2) * 2 * ny * nx * 16 + (ny * nx * 16 + my * nx * 16) \
        + (my * nx * 16 + 2 * mx * my * 4)
    pairs = (n_fft + 1) // 2
    return (fwd + pairs * inv if n_fft else 0) + n_direct * 8 * mx * my


def cpu_baseline_beside(c, ev, rhos, gamma, r, phi, a_min, n_kept, n_eval, fs_info=None):
    """The oracle timed on bounded samples of the stack, line-filter and simplex
    measurements (single-threaded numpy; oracle counts of 64 central ray rows)."""
    import numpy as np
    from oracle.lines import caustic_components, caustic_lines, line_filter_mirror32
    from oracle.simplex import line_chi2
    from oracle.maps import (map_scale, normalize_convolve_exact64_at, normalize_convolve_mirror32)
    from oracle.profiles import ld_pixel_weights
    from oracle.rays import rayshoot_mirror32_c

    win = c["window"]
    ny_r = c["rays"][5]
    counts, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], win, rows=(ny_r // 2 - 32, ny_r // 2 + 32),
                                    nthreads=max(1, min(CPU_WORKERS, os.cpu_count() or 1)))
    mx, my = win[4], win[5]
    d = win[2] / mx
    s32 = map_scale(c["rays"], win)
    t_stack, parts = 0.0, []
    for rho in rhos:
        w = ld_pixel_weights(rho, d, d, gamma)
        if np.count_nonzero(w) < STACK_FFT_MIN_TAPS and w.shape[0] <= 31:
            t = time.perf_counter()
            normalize_convolve_mirror32(counts, s32, w)
            dt = time.perf_counter() - t
            parts.append(f"rho {rho:.3g}: whole map {dt:.2f} s")
        else:
            px = [(my // 2 + 3 * k, mx // 2 - 5 * k) for k in range(8)]
            t = time.perf_counter()
            normalize_convolve_exact64_at(counts, float(s32), w, px)
            dt = (time.perf_counter() - t) * mx * my / len(px)
            parts.append(f"rho {rho:.3g}: {len(px)} pixels, {dt:.0f} s scaled")
        t_stack += dt
    amap = normalize_convolve_mirror32(counts, s32, ld_pixel_weights(c["rho"], d, d, 0.0))
    L = caustic_lines(caustic_components(c["s"], c["q"]), r, phi)
    n_sub = 128
    t = time.perf_counter()
    line_filter_mirror32(amap, win, L[:n_sub], a_min)
    t_filter = (time.perf_counter() - t) * len(L) / n_sub
    from oracle.lines import line_peaks_mirror32
    fs = None
    if fs_info is not None:
        from oracle.fsmag import critical_points_and_caustic, fs_magnification
        tr, tri, nreg = fs_info["truth"], fs_info["trial"], fs_info["nreg_trial"]
        tau = fs_info["zeta"]
        zs = (tau * math.cos(tri["alpha"]) - tri["u0"] * math.sin(tri["alpha"])) + \
            1j * (tau * math.sin(tri["alpha"]) + tri["u0"] * math.cos(tri["alpha"]))
        crit = critical_points_and_caustic(c["s"], c["q"], 1024)
        near_i = np.flatnonzero(nreg > 0)[:: max(1, int((nreg > 0).sum()) // 4)][:4]
        far_i = np.flatnonzero(nreg == -1)[:200]
        t = time.perf_counter()
        for k in near_i:
            fs_magnification(zs[k], tr["rho"], STACK_GAMMA, c["s"], c["q"], crit=crit)
        t_near = (time.perf_counter() - t) / max(len(near_i), 1)
        t = time.perf_counter()
        for k in far_i:
            fs_magnification(zs[k], tr["rho"], STACK_GAMMA, c["s"], c["q"], crit=crit)
        t_far = (time.perf_counter() - t) / max(len(far_i), 1)
        t_lc = t_near * int((nreg > 0).sum()) + t_far * int((nreg == -1).sum())
        fs = {"value": len(nreg) / t_lc, "unit": "epochs/s", "cores": 1, "kind": "oracle",
              "sample": f"caustic-crossing trial light curve: {len(near_i)} image-centred and "
                        f"{len(far_i)} point-source epochs, scaled to its "
                        f"{int((nreg > 0).sum())} and {int((nreg == -1).sum())} ({t_lc:.0f} s "
                        f"scaled)"}
    t = time.perf_counter()
    line_peaks_mirror32(amap, win, L[:n_sub], 0.2, 8)
    t_peaks = (time.perf_counter() - t) * len(L) / n_sub
    n_sx = 20  # chi-square evaluations timed; the simplex makes n_eval of them
    t = time.perf_counter()
    for k in range(n_sx):
        line_chi2(amap, win, ev["tt"], ev["F"], ev["w"], ev["t_ref"], L[k], (0.5 * k, math.log(20.0)))
    t_sx = (time.perf_counter() - t) * n_eval / n_sx
    return (
        {"value": len(rhos) / t_stack, "unit": "maps/s", "cores": 1, "kind": "oracle",
         "sample": "seven-radius stack of the oracle's counts (64 central ray rows), weights "
                   "computed beforehand: " + "; ".join(parts)},
        {"value": len(L) / t_filter, "unit": "lines/s", "cores": 1, "kind": "oracle",
         "sample": f"binary32 line filter of {n_sub} of {len(L)} lines ({t_filter:.1f} s scaled)"},
        {"value": n_kept / t_sx, "unit": "lines/s", "cores": 1, "kind": "oracle",
         "sample": f"{n_sx} chi-square evaluations of the oracle's simplex, scaled to the "
                   f"{n_eval} the GPU simplex made for {n_kept} lines ({t_sx:.0f} s scaled)"},
        {"value": len(L) / t_peaks, "unit": "lines/s", "cores": 1, "kind": "oracle",
         "sample": f"binary32 samples and peak scan of {n_sub} of {len(L)} lines "
                   f"({t_peaks:.1f} s scaled)"},
        fs,
    )


def leg_large(args, M, W, torch, np, dev):
    """Large single map (s = 0.8, q = 5e-3): 32768^2 rays into a 2048^2 map, rho = 2e-3
    disk convolution, the batched search of the 524288-trajectory grid against one
    3000-point light curve with its top 4096, and 50 L-BFGS rounds on those; steps
    serial and pipelined (the next step's map built on a second stream).  Beside it, on
    the step's counts and map: the seven-radius finite-source stack, the caustic-line
    filter and the line simplex."""
    stream = torch.cuda.Stream(device=dev)
    stream_a = torch.cuda.Stream(device=dev)
    ctx_b = M.Context.bound(stream)
    ctx_a = M.Context.bound(stream_a)
    c = W.config("large")
    ev = W.load_lightcurve("large")
    axes = W.grid_axes("large")
    n_traj = int(np.prod([len(a) for a in axes]))
    n_pts = len(ev["tt"])
    k = 4096
    rays_per_step = c["rays"][4] * c["rays"][5]
    evals_per_step = n_traj * n_pts
    with torch.cuda.stream(stream):
        lcs = M.LightCurveBatch.from_events([ev], dev)
        trajs = M.grid_trajectories(*axes)
        shape = (c["window"][5], c["window"][4])
        counts = torch.empty(shape, dtype=torch.int32, device=dev)
        amap = torch.empty(shape, dtype=torch.float32, device=dev)
        amap_build = torch.empty(shape, dtype=torch.float32, device=dev)
        maps = [(amap, c["window"])]
        M.rayshoot(c["s"], c["q"], c["rays"], c["window"], counts, ctx=ctx_b)
        M.normalize_convolve(counts, c["rays"], c["window"], c["rho"], out=amap, ctx=ctx_b)
        tuned = M.autotune(maps, lcs, trajs, ctx=ctx_b)
        sbuf = {}
        cand = (torch.empty((k, 4), dtype=torch.float64, device=dev),
                torch.empty(k, dtype=torch.int32, device=dev),
                torch.empty(k, dtype=torch.int32, device=dev))
        rbuf = (torch.empty(k, dtype=torch.float64, device=dev),
                torch.empty(k, dtype=torch.float64, device=dev))
        e_built, e_copied = torch.cuda.Event(), torch.cuda.Event()

        def build(pipelined, evs=None):
            if not pipelined:
                mark = (lambda j: evs[j].record(stream)) if evs else (lambda j: None)
                mark(0)
                M.rayshoot(c["s"], c["q"], c["rays"], c["window"], counts, ctx=ctx_b)
                mark(1)
                M.normalize_convolve(counts, c["rays"], c["window"], c["rho"], out=amap, ctx=ctx_b)
                mark(2)
                return
            mark = (lambda j: evs[j].record(stream_a)) if evs else (lambda j: None)
            mark(0)
            M.rayshoot(c["s"], c["q"], c["rays"], c["window"], counts, ctx=ctx_a)
            stream_a.wait_event(e_copied)
            mark(1)
            M.normalize_convolve(counts, c["rays"], c["window"], c["rho"], out=amap_build, ctx=ctx_a)
            mark(2)
            e_built.record(stream_a)

        def take_map():
            stream.wait_event(e_built)
            amap.copy_(amap_build)
            e_copied.record(stream)

        def solve(evs=None):
            mark = (lambda j: evs[j].record(stream)) if evs else (lambda j: None)
            mark(3)
            r = M.search(maps, lcs, trajs, "batched", chi2=False, top_k=k, out=sbuf, ctx=ctx_b)
            sbuf.update(r)
            mark(4)
            P, e_idx, m_idx = M.candidates_from_topk(trajs, r["topk_idx"], 1, out=cand, ctx=ctx_b)
            M.refine(maps, lcs, P, e_idx, m_idx, steps=50, inplace=True, chi2_out=rbuf, ctx=ctx_b)
            mark(5)

        def run(n, pipelined, ev_sets=None):
            evs = (lambda i: ev_sets[i]) if ev_sets else (lambda i: None)
            if not pipelined:
                for i in range(n):
                    build(False, evs(i))
                    solve(evs(i))
                return
            build(True, evs(0))
            for i in range(n):
                take_map()
                if i + 1 < n:
                    build(True, evs(i + 1))
                solve(evs(i))

        def timed(n, pipelined):
            ev_sets = [events_timer(torch, 6) for _ in range(n)]
            t0, t1 = events_timer(torch, 2)
            torch.cuda.synchronize()
            t0.record(stream_a if pipelined else stream)
            run(n, pipelined, ev_sets)
            t1.record(stream)
            torch.cuda.synchronize()
            stage = np.mean([[e[j].elapsed_time(e[j + 1]) for j in (0, 1, 3, 4)] for e in ev_sets],
                            axis=0)
            return t0.elapsed_time(t1) / n, stage

        progress("large: warm-up")
        run(1, False)
        run(1, True)
        n = max(1, args.large_steps)
        progress(f"large: {n} serial + {n} pipelined steps")
        serial_ms, stage = timed(n, False)
        pipe_ms, _ = timed(n, True)
        rec = {"workload": "large: s=0.8 q=5e-3, 32768^2 rays -> 2048^2 map, rho=2e-3, 3000-point "
                           "light curve, 524288-trajectory grid, top-4096 + 50 L-BFGS rounds",
               "serial_ms_per_step": serial_ms, "pipelined_ms_per_step": pipe_ms,
               "autotuned_search_shape": tuned,
               "stages_ms": dict(zip(("rayshoot", "normalize_convolve", "search_batched",
                                      "candidates_refine"), stage)),
               "rays_per_s": rays_per_step / (stage[0] * 1e-3),
               "search_point_evals_per_s_batched": evals_per_step / (stage[2] * 1e-3),
               "adjoint_point_evals_per_s_upper": 51 * k * n_pts / (stage[3] * 1e-3)}

        # Finite-source stack of the step's counts: seven radii log-spaced over [0.001, 1]
        # with limb-darkening coefficient 0.53.
        progress("large: finite-source stack")
        rhos = np.logspace(-3.0, 0.0, 7)
        sout = M.convolve_stack(counts, c["rays"], c["window"], rhos, STACK_GAMMA, ctx=ctx_b)
        torch.cuda.synchronize()
        e0, e1 = events_timer(torch, 2)
        e0.record(stream)
        for _ in range(5):
            M.convolve_stack(counts, c["rays"], c["window"], rhos, STACK_GAMMA, out=sout, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        st_ms = e0.elapsed_time(e1) / 5
        d = c["window"][2] / c["window"][4]
        fft_r = [r for r in rhos if math.ceil(r / d + 0.5) > 15 or
                 np.count_nonzero(M.profile_weights(r, d, d, STACK_GAMMA)) >= STACK_FFT_MIN_TAPS]
        mx, my = c["window"][4], c["window"][5]
        r_fft = max([math.ceil(r / d + 0.5) for r in fft_r], default=0)
        nfx = 1 << max(1, (mx + 2 * r_fft - 1).bit_length())
        nfy = 1 << max(1, (my + 2 * r_fft - 1).bit_length())
        sb = stack_bytes(mx, my, nfx, nfy, len(fft_r), len(rhos) - len(fft_r))
        rec["rho_stack"] = {
            "radii": [float(r) for r in rhos], "gamma": STACK_GAMMA, "ms": st_ms,
            "maps_per_s": len(rhos) / (st_ms * 1e-3), "fft_radii": len(fft_r),
            "map": [my, mx], "fft_size": [nfy, nfx],
            "roofline": {"bound": "hbm", "achieved": sb / (st_ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": sb / (st_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_call": sb,
                         "traffic": None,
                         "note": "algorithmic bytes of the whole call (transform passes, "
                                 "products, stores, direct radii) over the call's time"}}

        # Caustic-centred lines (sec. 4.2) through the minimum-magnification filter
        # (sec. 4.3) on the step's map, then the downhill simplex of every kept line.
        progress("large: caustic-line filter and line simplex")
        caus = M.caustics(c["s"], c["q"])
        r_ax, phi = np.linspace(0.0, 4.0, 32), np.linspace(0.0, 2 * np.pi, 257)[:-1]
        L = M.caustic_lines(caus, r_ax, phi)
        dl = torch.from_numpy(L).to(dev)
        Fv = np.asarray(ev["F"])
        a_min = 0.9 * float(Fv.max() / Fv.min())
        _, _, kept = M.line_filter(amap, c["window"], dl, a_min, ctx=ctx_b)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            M.line_filter(amap, c["window"], dl, a_min, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        lf_ms = e0.elapsed_time(e1) / 5
        w = c["window"]
        ns = math.ceil(2.0 * 0.5 * math.hypot(w[2], w[3]) * max(w[4] / w[2], w[5] / w[3])) + 1
        f_ops = sum(OPS_PER_FILTER_SAMPLE) * len(L) * ns / (lf_ms * 1e-3) / 1e12
        fpk = peak_for(OPS_PER_FILTER_SAMPLE) / 1e12
        lines_rec = {"caustics": int(len(caus)), "lines": int(len(L)), "kept": int(len(kept)),
                     "a_min": a_min, "samples_per_line": ns, "filter_ms": lf_ms,
                     "samples_per_s": len(L) * ns / (lf_ms * 1e-3),
                     "roofline": {"bound": "alu", "achieved": f_ops, "peak": fpk,
                                  "unit": "TFLOP/s", "frac": f_ops / fpk,
                                  "ops_per_unit_f32_f64": OPS_PER_FILTER_SAMPLE, "traffic": None,
                                  "note": "tera lane-operations/s over the whole call (packing "
                                          "the map and the compaction included)"}}
        # peak library + peak-count rejection (sec. 4.3, third optimisation) on the same
        # lines, and the simplex starts from the light curve's peak time (Eq. 7)
        pk_h, pk_min = 0.2, 2
        pk = M.line_peaks(amap, c["window"], dl, a_min, pk_min, pk_h, 8, ctx=ctx_b)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            pk = M.line_peaks(amap, c["window"], dl, a_min, pk_min, pk_h, 8, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        pk_ms = e0.elapsed_time(e1) / 5
        tp = float(ev["t"][int(np.argmax(Fv))])
        e0.record(stream)
        pst = M.peak_starts(dl, pk[5], pk[1], pk[2], pk[3], [tp], 20.0, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        lines_rec["peaks"] = {"hysteresis": pk_h, "min_peaks": pk_min, "ms": pk_ms,
                              "lines_per_s": len(L) / (pk_ms * 1e-3),
                              "samples_per_s": len(L) * ns / (pk_ms * 1e-3),
                              "kept": int(len(pk[5])),
                              "peaks_mean": float(pk[1].double().mean()),
                              "starts_ms": e0.elapsed_time(e1),
                              "starts_finite": int(torch.isfinite(pst[:, 0]).sum())}
        kl = dl[kept].contiguous()
        st0 = torch.tensor([[0.0, 20.0]], dtype=torch.float64, device=dev).repeat(len(kl), 1)
        sx_opts = dict(max_iter=5000, step_t0=2.0, step_ln_tE=0.2, ftol=1e-10)
        M.line_simplex(maps, lcs, kl, st0, ctx=ctx_b, **sx_opts)
        torch.cuda.synchronize()
        e0.record(stream)
        sx = M.line_simplex(maps, lcs, kl, st0, ctx=ctx_b, **sx_opts)
        e1.record(stream)
        torch.cuda.synchronize()
        sx_ms = e0.elapsed_time(e1)
        its = sx[3].double()
        n_eval = int(sx[4].long().sum())
        s_ops = sum(OPS_PER_SIMPLEX_POINT) * n_eval * n_pts / (sx_ms * 1e-3) / 1e12
        spk = peak_for(OPS_PER_SIMPLEX_POINT) / 1e12
        lines_rec["simplex"] = {
            "lines": int(len(kl)), "ms": sx_ms, "max_iter": 5000,
            "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
            "chi2_evaluations": n_eval, "best_chi2": float(sx[0].min()),
            "simplex_iterations_per_s": float(its.sum()) / (sx_ms * 1e-3),
            "point_evals_per_s": n_eval * n_pts / (sx_ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": s_ops, "peak": spk, "unit": "TFLOP/s",
                         "frac": s_ops / spk, "ops_per_unit_f32_f64": OPS_PER_SIMPLEX_POINT,
                         "traffic": None,
                         "note": "lines start in descending order of their peak; the longest simplex "
                                 "(iterations_max) sets the tail"}}
        rec["caustic_lines"] = lines_rec

        # Finite-source magnification without maps (sec. 5): the light curve's epochs on
        # its true trajectory, uniform disk of the true radius, image-centred ray shooting
        # within 10 rho of the caustic and the point source elsewhere
        progress("large: image-centred finite-source light curve")
        tr = ev["truth"]
        fs_params = (tr["t0"], tr["u0"], tr["tE"], tr["alpha"])
        td = torch.from_numpy(np.ascontiguousarray(ev["t"], dtype=np.float64)).to(dev)
        zeta = M.trajectory_positions(fs_params, td, ctx=ctx_b)
        A_fs, nreg = M.fs_magnification(c["s"], c["q"], zeta, tr["rho"], 0.0, ctx=ctx_b)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            zeta = M.trajectory_positions(fs_params, td, ctx=ctx_b)
            A_fs, nreg = M.fs_magnification(c["s"], c["q"], zeta, tr["rho"], 0.0, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        fs_ms = e0.elapsed_time(e1) / 3
        with np.load(W.golden_path("large")) as z:
            amag = np.asarray(z["e0"], dtype=np.float64)
        A_np, nr_np = A_fs.cpu().numpy(), nreg.cpu().numpy()
        rel = np.abs(A_np / amag - 1)
        rec["fs_lightcurve"] = {"epochs": int(len(A_np)), "rho": tr["rho"], "gamma": 0.0,
                                "ms": fs_ms, "epochs_per_s": len(A_np) / (fs_ms * 1e-3),
                                "image_centred_epochs": int((nr_np > 0).sum()),
                                "point_source_epochs": int((nr_np == -1).sum()),
                                "failed_epochs": int((nr_np < -1).sum()),
                                "grid": [512, 512],
                                "vs_synthesis_max_rel": float(rel.max()),
                                "vs_synthesis_median_rel": float(np.median(rel)),
                                "note": "synthesis magnifications: the oracle's quintic disk "
                                        "average within 10 rho of the caustic (quadrature), "
                                        "the point source elsewhere"}
        # a trial through the central caustic (u0 = 0), limb-darkened: the image-centred
        # branch at the caustic crossings
        trial = (tr["t0"], 0.0, tr["tE"], tr["alpha"])
        zt = M.trajectory_positions(trial, td, ctx=ctx_b)
        A_t, nreg_t = M.fs_magnification(c["s"], c["q"], zt, tr["rho"], STACK_GAMMA, ctx=ctx_b)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            zt = M.trajectory_positions(trial, td, ctx=ctx_b)
            A_t, nreg_t = M.fs_magnification(c["s"], c["q"], zt, tr["rho"], STACK_GAMMA, ctx=ctx_b)
        e1.record(stream)
        torch.cuda.synchronize()
        tr_ms = e0.elapsed_time(e1) / 3
        nt = nreg_t.cpu().numpy()
        # the image-centred integration's lens-equation samples: at most 1 + n_shrink
        # passes of n_theta x (n_r + 1) per region (the library's defaults)
        fs_samples = float(nt[nt > 0].sum()) * (1 + FS_SHRINK) * FS_THETA * (FS_R + 1)
        f_ops = fs_samples * sum(OPS_PER_FS_SAMPLE) / (tr_ms * 1e-3) / 1e12
        f_pk = peak_for(OPS_PER_FS_SAMPLE) / 1e12
        rec["fs_lightcurve"]["caustic_crossing_trial"] = {
            "params_t0_u0_tE_alpha": list(trial), "gamma": STACK_GAMMA, "ms": tr_ms,
            "epochs_per_s": len(nt) / (tr_ms * 1e-3), "image_centred_epochs": int((nt > 0).sum()),
            "regions": int(nt[nt > 0].sum()),
            "point_source_epochs": int((nt == -1).sum()), "failed_epochs": int((nt < -1).sum()),
            "A_max": float(A_t.max()),
            "roofline": {"bound": "alu", "achieved": f_ops, "peak": f_pk, "unit": "TFLOP/s",
                         "frac": f_ops / f_pk, "ops_per_unit_f32_f64": OPS_PER_FS_SAMPLE,
                         "ops_are_upper_bound": True, "traffic": None,
                         "note": "tera lane-operations/s of the image-centred integration's "
                                 "lens-equation samples (at most 1 + n_shrink passes per region) "
                                 "over the whole light-curve call, which also classifies the "
                                 "epochs, solves the far ones and builds the regions"}}
        fs_info = dict(zeta=(np.asarray(ev["t"]) - tr["t0"]) / tr["tE"], nreg=nr_np, truth=tr,
                       trial=dict(tr, u0=0.0), nreg_trial=nt)
        beside = dict(c=c, ev=ev, rhos=rhos, gamma=STACK_GAMMA, r=r_ax, phi=phi, a_min=a_min, fs=fs_info,
                      n_kept=int(len(kl)), n_eval=n_eval)
    del counts, amap, amap_build
    torch.cuda.empty_cache()
    return rec, beside


def main():
    args = parse()
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace)
    if args.summarize_pmc:
        return summarize_pmc(args.summarize_pmc)
    if args.copy_bytes:
        return copy_kernel(args.copy_bytes)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(on several GPUs the path would deal maps or ray rows to GPUs and gather "
              "the per-GPU top-k lists)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import workloads as W

    # the oracle's baseline first, before anything touches the GPU (its workers fork)
    cpu = None
    if not args.no_cpu_baseline:
        cb, cr = W.config("batched"), W.config("refine")
        n_pts = np.array([t["npts"] for t in W.truths("batched")])
        nb = len(W.map_bank("batched"))
        units = {"rays": nb * (cb["rays"][4] * cb["rays"][5] + cr["rays"][4] * cr["rays"][5]),
                 "pixels": nb * (cb["window"][4] * cb["window"][5] + cr["window"][4] * cr["window"][5]),
                 "evals": int(n_pts.sum()) * nb * cb["n_traj"],
                 "cand_round_points": (cr["steps"] + 1) * cr["top_k"] * int(n_pts[:cr["n_events"]].sum())}
        cpu = cpu_baseline_batched(units)

    import torch

    import paper_1511_01157_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    head = leg_batched(args, M, W, torch, np, dev)
    sq = None if args.no_sqgrid else leg_sqgrid(args, M, W, torch, np, dev)
    large, beside = (None, None) if args.no_large else leg_large(args, M, W, torch, np, dev)
    if cpu is not None and beside is not None:
        progress("cpu baseline beside the large workload (stack, line filter, simplex)")
        b_st, b_lf, b_sx, b_pk, b_fs = cpu_baseline_beside(
            beside["c"], beside["ev"], beside["rhos"], beside["gamma"], beside["r"], beside["phi"],
            beside["a_min"], beside["n_kept"], beside["n_eval"], beside.get("fs"))
        large["rho_stack"]["cpu_baseline"] = b_st
        large["caustic_lines"]["cpu_baseline"] = b_lf
        large["caustic_lines"]["simplex"]["cpu_baseline"] = b_sx
        large["caustic_lines"]["peaks"]["cpu_baseline"] = b_pk
        if b_fs is not None:
            large["fs_lightcurve"]["caustic_crossing_trial"]["cpu_baseline"] = b_fs

    dom = head["dominant"]
    line = {
        "metric": "light-curve point-evals/s (chi2 search) + rays/s (map build); batched vs plain",
        "value": head["value"], "unit": "point-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, f64 sums",
        "data": "synthetic (seeded light curves, oracle-computed magnifications)",
        "config": head["config"],
        "stages_ms": head["stages_ms"],
        "rays_per_s": head["rays_per_s"],
        "search_point_evals_per_s": head["search_point_evals_per_s"],
        "adjoint_point_evals_per_s_upper": head["adjoint_point_evals_per_s_upper"],
        "refine_chi2_not_raised": head["refine_chi2_not_raised"],
        "refine_chi2_lowered": head["refine_chi2_lowered"],
        "wall_s_timed": head["wall_s_timed"],
        "roofline": dict(head["kernels"][dom], op_note=OP_NOTE,
                         kernel_ms_per_step=head["kernel_ms_per_step"]),
        "kernels": head["kernels"],
        "sqgrid": sq,
        "large": large,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
