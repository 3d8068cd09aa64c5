// Trajectory search on gfx950 (sec. 4.2 of McDougall & Albrow 2015: the chi-square of
// every trajectory through a map, sampled by bilinear interpolation; Eqs. 5-6: the flux
// is linear in the magnification, so (F_s, F_b) are profiled out by weighted least
// squares).
//
// Layout.  One wavefront scores TU neighbouring trajectories at a time: its 64 lanes
// stride over the light-curve points (time-ordered, so a wave's lanes sample
// neighbouring map cells and leave the map together), each lane keeps FP64 partial
// sums of the normal equations in centred form (b = A - 1 against the mean-centred
// weighted flux) per trajectory, and a fixed-order reduction (bitwise the butterfly of
// each value) totals them.  S_w, the weighted mean flux and V = sum w (F - Fbar)^2
// depend only on the light curve and are computed once per event.  The 2x2 solve gives
// chi2 = V - F_s C in the same pass; when the rounding bound of that form exceeds 1e-9
// relative (ill-conditioned or near-perfect fits) the wave re-samples and sums
// w (F - F_s A - F_b)^2 directly.
//
// Plain mode launches one grid per (event, map), one trajectory per wavefront.  Batched
// mode launches one persistent grid whose wavefronts pull (map, event, trajectory
// group) items from per-XCD work queues, so thousands of (event, map) pairs of uneven
// length share one launch; the per-trajectory arithmetic and reduction order are the
// same, so results are bitwise identical between the modes.

#include "internal.h"

#include <algorithm>

namespace morse {

namespace {

// ---------------------------------------------------------------------------
// Light-curve preparation, one workgroup per event: S_w and S_F with
// Neumaier-compensated partial sums combined by a fixed pairwise tree, Fbar = S_F/S_w, then
// wFc = w (F - Fbar) per point and V = sum w (F - Fbar)^2 the same way.

// Pairwise tree over the workgroup's Neumaier partials (sum, compensation) held in
// columns (2q, 2q + 1) of s_part, q < NQ, in a fixed order; every thread returns the
// totals.
template <int NQ>
__device__ __forceinline__ void tree_totals(double (*s_part)[4], double (&tot)[NQ]) {
  const int tid = threadIdx.x;
  for (int half = blockDim.x / 2; half >= 1; half >>= 1) {
    if (tid < half) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        double sm = s_part[tid][2 * q], c = s_part[tid][2 * q + 1];
        neumaier_add(sm, c, s_part[tid + half][2 * q]);
        s_part[tid][2 * q] = sm;
        s_part[tid][2 * q + 1] = c + s_part[tid + half][2 * q + 1];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) tot[q] = s_part[0][2 * q] + s_part[0][2 * q + 1];
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_lc_prep(const double* __restrict__ F,
                                                 const double* __restrict__ w,
                                                 const int64_t* __restrict__ off,
                                                 double* __restrict__ wFc, double* __restrict__ sums) {
  __shared__ double s_part[256][4];
  const int e = blockIdx.x;
  const int64_t a = off[e], b = off[e + 1];
  double s0 = 0, c0 = 0, s1 = 0, c1 = 0;
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    const double wi = w[i];
    neumaier_add(s0, c0, wi);
    neumaier_add(s1, c1, wi * F[i]);
  }
  s_part[threadIdx.x][0] = s0;
  s_part[threadIdx.x][1] = c0;
  s_part[threadIdx.x][2] = s1;
  s_part[threadIdx.x][3] = c1;
  __syncthreads();
  double t01[2];
  tree_totals<2>(s_part, t01);
  const double Sw = t01[0];
  const double Fbar = t01[1] / Sw;
  double s2 = 0, c2 = 0;
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    const double d = F[i] - Fbar;
    const double wd = w[i] * d;
    wFc[i] = wd;
    neumaier_add(s2, c2, wd * d);
  }
  s_part[threadIdx.x][0] = s2;
  s_part[threadIdx.x][1] = c2;
  __syncthreads();
  double t2[1];
  tree_totals<1>(s_part, t2);
  if (threadIdx.x == 0) {
    sums[3 * e] = Sw;
    sums[3 * e + 1] = Fbar;
    sums[3 * e + 2] = t2[0];
  }
}

// Per-trajectory constants: FP64 trigonometry, rounded once to binary32.
__device__ __forceinline__ TrajC make_traj(double t0, double u0, double tE, double al) {
  double s, c;
  sincos(al, &s, &c);
  TrajC r;
  r.t0 = t0;
  r.iE = (float)(1.0 / tE);
  r.ca = (float)c;
  r.sa = (float)s;
  r.bx = (float)(-u0 * s);
  r.by = (float)(u0 * c);
  r.pad = 0.0f;
  return r;
}

__global__ void k_traj_prep_list(const double* __restrict__ params, int64_t n, TrajC* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double* p = params + 4 * i;
    out[i] = make_traj(p[0], p[1], p[2], p[3]);
  }
}

// axes = [u0 (nu) | alpha (na) | t0 (nt) | tE (ne)]; index ((iu*na + ia)*nt + it)*ne + ie
__global__ void k_traj_prep_grid(const double* __restrict__ axes, int32_t nu, int32_t na, int32_t nt,
                                 int32_t ne, TrajC* __restrict__ out) {
  const int64_t n = (int64_t)nu * na * nt * ne;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = i;
    const int ie = (int)(r % ne);
    r /= ne;
    const int it = (int)(r % nt);
    r /= nt;
    const int ia = (int)(r % na);
    const int iu = (int)(r / na);
    out[i] = make_traj(axes[nu + na + it], axes[iu], axes[nu + na + nt + ie], axes[nu + ia]);
  }
}

// ---------------------------------------------------------------------------
// Score TU trajectories with one wavefront.  All lanes return the same values.
// Each lane takes the points lane, lane + 64, ... in order; the TU trajectories' cells
// are all located and requested before the first is blended, so a wavefront has TU
// gathers in flight at a time.  A lane off the map requests cell 0 and takes the
// single-lens branch.  With TU >= 4 registers set the occupancy, so the loop keeps
// fewer live: no load of the next point ahead, and the single-lens branch recomputes
// the source position from tau (the same operations, so the same bits) rather than
// keeping it across the gathers; six wavefronts then fit on a SIMD where four did.  With fewer trajectories per wavefront the next point's light-curve values
// are loaded while the current one is scored.  Every trajectory's sums see the
// points in the same order for any TU, and wave_sums reduces each over the butterfly
// tree, so the results do not depend on TU.  Arrays are addressed by 32-bit offsets
// from uniform bases.
template <int TU>
__device__ __forceinline__ void score_group(const MapC& m, const float* __restrict__ t,
                                            const double* __restrict__ w,
                                            const double* __restrict__ wFc,
                                            const double* __restrict__ F, int32_t np, double Sw,
                                            double Fbar, double V, const float (&t0p)[TU],
                                            const TrajC (&c)[TU], int lane, double (&chi2)[TU],
                                            double (&Fs)[TU], double (&Fb)[TU]) {
  constexpr bool kLean = TU >= 4;
  double acc[3 * TU];  // (B1, B2, C) per trajectory
#pragma unroll
  for (int q = 0; q < 3 * TU; ++q) acc[q] = 0.0;
  // the point (tt, wv, fv) for the TU trajectories
  auto add_point = [&](float tt, double wv, double fv) {
    Loc l[TU];
    Quad cell[TU];
#pragma unroll
    for (int v = 0; v < TU; ++v)
      l[v] = locate(m, tt, t0p[v], c[v].iE, c[v].ca, c[v].sa, c[v].bx, c[v].by);
#pragma unroll
    for (int v = 0; v < TU; ++v) cell[v] = ldq(m, l[v].q);
#pragma unroll
    for (int v = 0; v < TU; ++v) {
      float A = 0.0f;
      // with TU >= 4 a wavefront whose lanes are all off the map skips the interpolation
      if (!kLean || __builtin_amdgcn_ballot_w64(l[v].on) != 0) {
        const float e0 = cell[v].v10 - cell[v].v00, e1 = cell[v].v11 - cell[v].v01;
        const float ax0 = cell[v].v00 + l[v].fx * e0, ax1 = cell[v].v01 + l[v].fx * e1;
        A = ax0 + l[v].fy * (ax1 - ax0);
      }
      if (!l[v].on) {
        if constexpr (kLean) {
          float tau = l[v].tau;
          asm volatile("" : "+v"(tau));  // opaque copy: the compiler cannot reuse locate's zx, zy
          A = point_lens_A(tau * c[v].ca + c[v].bx, tau * c[v].sa + c[v].by);
        } else {
          A = point_lens_A(l[v].zx, l[v].zy);
        }
      }
      const double b = (double)A - 1.0;
      const double wb = wv * b;
      acc[3 * v] += wb;
      acc[3 * v + 1] = fma(wb, b, acc[3 * v + 1]);
      acc[3 * v + 2] = fma(b, fv, acc[3 * v + 2]);
    }
  };
  if constexpr (kLean) {
    for (int32_t i0 = lane; i0 < np; i0 += kWave)
      add_point(ldg(t, (uint32_t)i0), ldg(w, (uint32_t)i0), ldg(wFc, (uint32_t)i0));
  } else {  // the next point's light-curve values are loaded while this one is scored
    uint32_t in = (uint32_t)min(lane, np - 1);
    float tn = ldg(t, in);
    double wn = ldg(w, in), fn = ldg(wFc, in);
    for (int32_t i0 = lane; i0 < np; i0 += kWave) {
      const float tt = tn;
      const double wv = wn, fv = fn;
      in = (uint32_t)min(i0 + kWave, np - 1);  // past the end: the last point, never used
      tn = ldg(t, in);
      wn = ldg(w, in);
      fn = ldg(wFc, in);
      add_point(tt, wv, fv);
    }
  }
  wave_sums<3 * TU>(acc);
#pragma unroll
  for (int v = 0; v < TU; ++v) {
    const Fit f = centred_fit(Sw, Fbar, V, acc[3 * v], acc[3 * v + 1], acc[3 * v + 2],
                              fit_terms(np, kWave));
    Fs[v] = f.Fs;
    Fb[v] = f.Fb;
    chi2[v] = f.chi2;
    if (f.recheck) {  // wave-uniform: the sums are identical on every lane
      double q = 0.0, qc = 0.0;
      for (int32_t i = lane; i < np; i += kWave) {
        const double a = (double)sample_A(m, ldg(t, (uint32_t)i), t0p[v], c[v].iE, c[v].ca,
                                          c[v].sa, c[v].bx, c[v].by);
        const double r = ldg(F, (uint32_t)i) - Fs[v] * a - Fb[v];
        neumaier_add(q, qc, (ldg(w, (uint32_t)i) * r) * r);
      }
      chi2[v] = wave_sum(q + qc);
    }
  }
}

__global__ __launch_bounds__(256) void k_search_plain(const TrajC* __restrict__ tc, int64_t n_traj,
                                                      LcView lc, int32_t e, MapC m, SearchOut out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wpb = blockDim.x / kWave;
  const int64_t nw = (int64_t)gridDim.x * wpb;
  const int64_t p0 = lc.off[e];
  const int32_t np = (int32_t)(lc.off[e + 1] - p0);
  const float* t = lc.t + p0;
  const double* w = lc.w + p0;
  const double* wFc = lc.wFc + p0;
  const double* F = lc.F + p0;
  const double Sw = lc.sums[3 * e], Fbar = lc.sums[3 * e + 1], V = lc.sums[3 * e + 2];
  const double tref = lc.t_ref[e];
  for (int64_t k = (int64_t)blockIdx.x * wpb + (threadIdx.x / kWave); k < n_traj; k += nw) {
    const TrajC c[1] = {tc[k]};
    const float t0p[1] = {(float)(c[0].t0 - tref)};
    double chi2[1], Fs[1], Fb[1];
    score_group<1>(m, t, w, wFc, F, np, Sw, Fbar, V, t0p, c, lane, chi2, Fs, Fb);
    if (lane == 0) {
      if (out.chi2) out.chi2[k] = chi2[0];
      if (out.fs) out.fs[k] = Fs[0];
      if (out.fb) out.fb[k] = Fb[0];
    }
  }
}

// Persistent batched search.  Every wavefront pulls its own work items (no workgroup
// barrier, so a slow trajectory never holds up other waves).  The item space is cut
// into kQueues contiguous ranges, one queue each; workgroups are dispatched to the 8
// XCDs in turn, so blockIdx % 8 names the workgroup's XCD and its home queue: each
// XCD's L2 serves one compact part of the work, and a wave whose queue is empty moves
// on to the next queue until all are drained.  Trajectories are taken in groups of
// TU neighbours, scored together.  Item = (map * n_events + event) * n_blocks + b
// scores groups b, b + n_blocks, ... (traj_per_item / TU of them): the waves of an
// XCD running at the same time take neighbouring items, so they score neighbouring
// trajectories of the same map and light curve.  On a product grid the scoring order
// runs over (alpha, u0, t0, tE), tE fastest, so neighbouring trajectories lie on
// nearly the same line through the map (the (u0, alpha, t0, tE) index order of the
// outputs is unchanged); trajectory lists are scored in the order of `perm`, grouped by
// direction, for the same reason.
// Trajectory index of scoring position p of event e (see k_search_batched).
__device__ __forceinline__ int64_t traj_of(const BatchedArgs& a, int64_t p, int32_t e) {
  if (a.na <= 0) {
    if (!a.perm) return p;
    const int64_t base = a.shared ? 0 : (int64_t)e * a.n_traj;  // perm holds indices over all lists
    return (int64_t)uniform(a.perm[base + p]) - base;
  }
  const uint32_t u = (uint32_t)p;  // n_traj < 2^31
  const uint32_t ie = u % (uint32_t)a.ne, r1 = u / (uint32_t)a.ne;
  const uint32_t it = r1 % (uint32_t)a.nt, r2 = r1 / (uint32_t)a.nt;
  const uint32_t iu = r2 % (uint32_t)a.nu, ia = r2 / (uint32_t)a.nu;
  return (((int64_t)iu * a.na + ia) * a.nt + it) * a.ne + ie;
}

template <int TU>
__global__ __launch_bounds__(512) void k_search_batched(BatchedArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t ng = (a.n_traj + TU - 1) / TU;
  const int64_t gpi = max(a.traj_per_item / TU, 1);
  const int64_t nb = (ng + gpi - 1) / gpi;
  const int64_t total = nb * a.n_events * a.n_maps;
  int q = blockIdx.x % kQueues;
  int left = kQueues;
  for (;;) {
    const int64_t lo = total * q / kQueues, hi = total * (q + 1) / kQueues;
    int rel32 = 0;
    if (lane == 0) rel32 = (int)atomicAdd(a.counter + q * kQueueStride, 1u);
    // first-lane read: the item is provably wave-uniform, so everything derived from it
    // (indices, map and trajectory constants) stays in scalar registers
    const int64_t item = lo + (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(rel32);
    if (item >= hi) {  // this queue is drained (and stays drained)
      if (--left == 0) break;
      q = (q + 1) % kQueues;
      continue;
    }
    const int64_t b = item % nb;
    const int64_t me = item / nb;
    const int32_t e = (int32_t)(me % a.n_events);
    const int32_t mi = (int32_t)(me / a.n_events);
    const MapC m = uniform(a.maps[mi]);
    const int64_t p0 = uniform(a.lc.off[e]);
    const int32_t np = (int32_t)(uniform(a.lc.off[e + 1]) - p0);
    const double Sw = uniform(a.lc.sums[3 * e]), Fbar = uniform(a.lc.sums[3 * e + 1]),
                 V = uniform(a.lc.sums[3 * e + 2]);
    const double tref = uniform(a.lc.t_ref[e]);
    const TrajC* tc = a.tc + (a.shared ? 0 : (int64_t)e * a.n_traj);
    const int64_t obase = ((int64_t)e * a.n_maps + mi) * a.n_traj;
    for (int64_t g = b; g < ng; g += nb) {
      TrajC c[TU];
      float t0p[TU];
      int64_t kk[TU];
#pragma unroll
      for (int v = 0; v < TU; ++v) {  // a short last group repeats its last trajectory
        kk[v] = traj_of(a, min(g * TU + v, a.n_traj - 1), e);
        c[v] = uniform(tc[kk[v]]);
        t0p[v] = (float)(c[v].t0 - tref);
      }
      double chi2[TU], Fs[TU], Fb[TU];
      score_group<TU>(m, a.lc.t + p0, a.lc.w + p0, a.lc.wFc + p0, a.lc.F + p0, np, Sw, Fbar, V,
                      t0p, c, lane, chi2, Fs, Fb);
      if (lane == 0) {
#pragma unroll
        for (int v = 0; v < TU; ++v) {
          const int64_t k = kk[v];
          if (g * TU + v < a.n_traj) {
            if (a.out.chi2) a.out.chi2[obase + k] = chi2[v];
            if (a.out.fs) a.out.fs[obase + k] = Fs[v];
            if (a.out.fb) a.out.fb[obase + k] = Fb[v];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Selection.  Keys order doubles totally: -0 is taken as +0, NaN after everything;
// ties broken by the index.
__device__ __forceinline__ uint64_t order_key(double x) {
  if (x != x) return ~0ull;
  if (x == 0.0) x = 0.0;
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_best(const double* __restrict__ chi2, int64_t seg_len,
                                              double* __restrict__ best_chi2,
                                              int64_t* __restrict__ best_idx) {
  __shared__ uint64_t s_key[4];
  __shared__ int64_t s_idx[4];
  const double* base = chi2 + (int64_t)blockIdx.x * seg_len;
  uint64_t bk = ~0ull;
  int64_t bi = INT64_MAX;
  for (int64_t i = threadIdx.x; i < seg_len; i += blockDim.x) {
    const uint64_t k = order_key(base[i]);
    if (k < bk || (k == bk && i < bi)) {
      bk = k;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t ok = __shfl_xor(bk, o, kWave);
    const int64_t oi = __shfl_xor(bi, o, kWave);
    if (ok < bk || (ok == bk && oi < bi)) {
      bk = ok;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    s_key[threadIdx.x >> 6] = bk;
    s_idx[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q)
      if (s_key[q] < bk || (s_key[q] == bk && s_idx[q] < bi)) {
        bk = s_key[q];
        bi = s_idx[q];
      }
    if (seg_len == 0) bi = -1;
    if (best_chi2) best_chi2[blockIdx.x] = (bi >= 0) ? base[bi] : __longlong_as_double(0x7ff8000000000000ll);
    if (best_idx) best_idx[blockIdx.x] = bi;
  }
}

// Top-k per segment by radix select over the composite key (order_key(chi2), index):
// 6 passes of 11-bit digits over the 64-bit key, then (only when the k-th key is shared
// by more items than remain to take) 3 passes over the 32-bit index among those ties.
// Each pass: every workgroup histograms its slice of the segment in LDS and merges it
// into the segment's global histogram with atomics; one workgroup per segment then
// scans the 2048 bins, fixes the next digit of the threshold and clears the histogram.
// A collect pass writes exactly k survivors (order-free atomic slots) and one
// workgroup per segment sorts them by (key, index) in LDS.
constexpr int TK_BINS = 2048;
constexpr int TK_THREADS = 256;
constexpr int TK_MAXK = 4096;
constexpr int TK_PASSES = 9;

struct TkState {
  uint64_t prefix;  // fixed high digits of the threshold key
  uint64_t mask;
  int64_t krem;     // rank still to place within the current bin
  int64_t bincount; // items in the chosen bin of the last pass
  uint32_t iprefix, imask;  // index digits (tie passes)
  int32_t need_idx;
  int32_t taken;    // collect counter
};

__device__ __forceinline__ void tk_digit(int pass, int& shift, int& width) {
  // key passes: bits 63..53, 52..42, 41..31, 30..20, 19..9, 8..0; index: 31..21, 20..10, 9..0
  const int sh[TK_PASSES] = {53, 42, 31, 20, 9, 0, 21, 10, 0};
  const int wd[TK_PASSES] = {11, 11, 11, 11, 11, 9, 11, 11, 10};
  shift = sh[pass];
  width = wd[pass];
}

__global__ void k_tk_init(TkState* st, uint32_t* hist, uint64_t* keys, uint32_t* idx,
                          int64_t n_seg, int64_t seg_len, int32_t k) {
  const int64_t seg = blockIdx.x;
  if (seg >= n_seg) return;
  for (int b = threadIdx.x; b < TK_BINS; b += blockDim.x) hist[seg * TK_BINS + b] = 0u;
  for (int b = threadIdx.x; b < k; b += blockDim.x) {  // unfilled slots read as invalid
    keys[seg * k + b] = ~0ull;
    idx[seg * k + b] = 0xffffffffu;
  }
  if (threadIdx.x == 0) {
    TkState s;
    s.prefix = 0;
    s.mask = 0;
    s.krem = min((int64_t)k, seg_len);
    s.bincount = 0;
    s.iprefix = 0;
    s.imask = 0;
    s.need_idx = 0;
    s.taken = 0;
    st[seg] = s;
  }
}

__global__ __launch_bounds__(TK_THREADS) void k_tk_hist(const double* __restrict__ chi2,
                                                        int64_t seg_len,
                                                        const TkState* __restrict__ st,
                                                        uint32_t* __restrict__ hist, int pass) {
  __shared__ uint32_t h[TK_BINS];
  const int64_t seg = blockIdx.y;
  const TkState s = st[seg];
  if (s.krem <= 0 || (pass >= 6 && !s.need_idx)) return;  // uniform per workgroup
  for (int b = threadIdx.x; b < TK_BINS; b += TK_THREADS) h[b] = 0u;
  __syncthreads();
  int shift, width;
  tk_digit(pass, shift, width);
  const uint32_t dmask = (1u << width) - 1u;
  const double* base = chi2 + seg * seg_len;
  for (int64_t i = blockIdx.x * (int64_t)TK_THREADS + threadIdx.x; i < seg_len;
       i += (int64_t)gridDim.x * TK_THREADS) {
    const uint64_t key = order_key(base[i]);
    if (pass < 6) {
      if ((key & s.mask) == s.prefix) atomicAdd(&h[(uint32_t)(key >> shift) & dmask], 1u);
    } else if (key == s.prefix && (((uint32_t)i) & s.imask) == s.iprefix) {
      atomicAdd(&h[((uint32_t)i >> shift) & dmask], 1u);
    }
  }
  __syncthreads();
  uint32_t* g = hist + seg * TK_BINS;
  for (int b = threadIdx.x; b < TK_BINS; b += TK_THREADS)
    if (h[b]) atomicAdd(&g[b], h[b]);
}

__global__ __launch_bounds__(TK_THREADS) void k_tk_pick(TkState* __restrict__ st,
                                                        uint32_t* __restrict__ hist, int pass) {
  __shared__ int64_t incl[TK_THREADS];
  const int64_t seg = blockIdx.x;
  TkState s = st[seg];
  if (s.krem <= 0 || (pass >= 6 && !s.need_idx)) return;
  uint32_t* g = hist + seg * TK_BINS;
  constexpr int PER = TK_BINS / TK_THREADS;
  const int t = threadIdx.x;
  uint32_t c[PER];
  int64_t part = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    c[q] = g[t * PER + q];
    part += c[q];
  }
  incl[t] = part;
  __syncthreads();
  for (int o = 1; o < TK_THREADS; o <<= 1) {
    const int64_t v = (t >= o) ? incl[t - o] : 0;
    __syncthreads();
    incl[t] += v;
    __syncthreads();
  }
  const int64_t before = incl[t] - part;
  int shift, width;
  tk_digit(pass, shift, width);
  if (before < s.krem && s.krem <= incl[t]) {
    int64_t cum = before;
    int d = t * PER;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (cum + c[q] >= s.krem) {
        d = t * PER + q;
        break;
      }
      cum += c[q];
    }
    const int64_t cnt = g[d];
    s.krem -= cum;
    s.bincount = cnt;
    const uint64_t wm = (1ull << width) - 1ull;
    if (pass < 6) {
      s.prefix |= (uint64_t)d << shift;
      s.mask |= wm << shift;
      if (pass == 5) s.need_idx = (s.bincount != s.krem) ? 1 : 0;
    } else {
      s.iprefix |= (uint32_t)d << shift;
      s.imask |= (uint32_t)wm << shift;
    }
    st[seg] = s;
  }
  __syncthreads();
  for (int b = t; b < TK_BINS; b += TK_THREADS) g[b] = 0u;
}

// Survivors: key < T, or key == T and (all ties taken, or index <= the chosen index).
__global__ __launch_bounds__(TK_THREADS) void k_tk_collect(const double* __restrict__ chi2,
                                                           int64_t seg_len, int32_t k,
                                                           TkState* __restrict__ st,
                                                           uint64_t* __restrict__ keys,
                                                           uint32_t* __restrict__ idx) {
  const int64_t seg = blockIdx.y;
  const TkState s = st[seg];
  const double* base = chi2 + seg * seg_len;
  for (int64_t i = blockIdx.x * (int64_t)TK_THREADS + threadIdx.x; i < seg_len;
       i += (int64_t)gridDim.x * TK_THREADS) {
    const uint64_t key = order_key(base[i]);
    bool take = key < s.prefix;
    if (key == s.prefix) take = !s.need_idx || ((uint32_t)i <= s.iprefix);
    if (take) {
      const int pos = atomicAdd(&st[seg].taken, 1);
      if (pos < k) {
        keys[seg * k + pos] = key;
        idx[seg * k + pos] = (uint32_t)i;
      }
    }
  }
}

// Final order of the k selected (key, index) pairs of a segment by rank: element e
// goes to position #{(key, index) < (key_e, index_e)} (the pairs are distinct, so the
// ranks are a permutation).  A workgroup stages the segment's pairs in LDS and ranks
// TKR_ELEMS of them, TKR_SPLIT threads per element each counting over a slice of the
// pairs (a whole wavefront reads the same LDS words at once; the loop is unrolled so
// the reads overlap).  Positions past the segment's length get index -1 and NaN.
constexpr int TKR_ELEMS = 16;
constexpr int TKR_SPLIT = 16;
__global__ __launch_bounds__(TKR_ELEMS * TKR_SPLIT) void k_tk_rank(
    const double* __restrict__ chi2, int64_t seg_len, int32_t k,
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx,
    double* __restrict__ out_chi2, int64_t* __restrict__ out_idx) {
  __shared__ uint64_t lk[TK_MAXK];
  __shared__ uint32_t li[TK_MAXK];
  __shared__ uint32_t part[TKR_SPLIT][TKR_ELEMS];
  const int64_t seg = blockIdx.y;
  const int tid = threadIdx.x;
  const int keff = (int)min((int64_t)k, seg_len);
  for (int q = tid; q < keff; q += blockDim.x) {
    lk[q] = keys[seg * k + q];
    li[q] = idx[seg * k + q];
  }
  __syncthreads();
  const int el = tid % TKR_ELEMS, slice = tid / TKR_ELEMS;
  const int e = blockIdx.x * TKR_ELEMS + el;
  uint32_t count = 0;
  if (e < keff) {
    const uint64_t mk = lk[e];
    const uint32_t mi = li[e];
    const int j0 = (int)((int64_t)keff * slice / TKR_SPLIT);
    const int j1 = (int)((int64_t)keff * (slice + 1) / TKR_SPLIT);
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
      const uint64_t kj = lk[j];
      const uint32_t ij = li[j];
      count += (kj < mk || (kj == mk && ij < mi)) ? 1u : 0u;
    }
  }
  part[slice][el] = count;
  __syncthreads();
  if (slice != 0 || e >= k) return;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  if (e < keff) {
    uint32_t rank = 0;
#pragma unroll
    for (int q = 0; q < TKR_SPLIT; ++q) rank += part[q][el];
    const uint32_t ie = li[e];
    const bool valid = (int64_t)ie < seg_len;
    out_idx[seg * k + rank] = valid ? (int64_t)ie : -1;
    out_chi2[seg * k + rank] = valid ? chi2[seg * seg_len + ie] : nan;
  } else {
    out_idx[seg * k + e] = -1;
    out_chi2[seg * k + e] = nan;
  }
}

// Top-k flat index -> (t0, u0, tE, alpha), event and map index.  axes != nullptr:
// product grid [u0 | alpha | t0 | tE]; else list rows (per event unless shared).
__global__ void k_candidates(const double* __restrict__ axes, int32_t nu, int32_t na, int32_t nt,
                             int32_t ne, const double* __restrict__ list, int32_t shared,
                             int64_t n_traj, int32_t n_events, int32_t n_maps, int32_t k,
                             const int64_t* __restrict__ idx, double* __restrict__ params,
                             int32_t* __restrict__ event, int32_t* __restrict__ mapidx) {
  const int64_t n = (int64_t)n_events * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = (int32_t)(i / k);
    int64_t f = idx[i];
    if (f < 0 || f >= (int64_t)n_maps * n_traj) f = 0;
    const int32_t m = (int32_t)(f / n_traj);
    const int64_t tj = f - (int64_t)m * n_traj;
    double* out = params + 4 * i;
    if (axes) {
      int64_t r = tj;
      const int ie = (int)(r % ne);
      r /= ne;
      const int it = (int)(r % nt);
      r /= nt;
      const int ia = (int)(r % na);
      const int iu = (int)(r / na);
      out[0] = axes[nu + na + it];
      out[1] = axes[iu];
      out[2] = axes[nu + na + nt + ie];
      out[3] = axes[nu + ia];
    } else {
      const double* p = list + 4 * ((shared ? 0 : (int64_t)e * n_traj) + tj);
      out[0] = p[0];
      out[1] = p[1];
      out[2] = p[2];
      out[3] = p[3];
    }
    event[i] = e;
    mapidx[i] = m;
  }
}

}  // namespace

hipError_t launch_candidates(const double* axes, int32_t nu, int32_t na, int32_t nt, int32_t ne,
                             const double* list, int32_t shared, int64_t n_traj, int32_t n_events,
                             int32_t n_maps, int32_t k, const int64_t* idx, double* params,
                             int32_t* event, int32_t* mapidx, hipStream_t st) {
  const int64_t n = (int64_t)n_events * k;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_candidates, dim3((unsigned)blocks), dim3(256), 0, st, axes, nu, na, nt, ne,
                     list, shared, n_traj, n_events, n_maps, k, idx, params, event, mapidx);
  return hipGetLastError();
}

hipError_t launch_lc_prep(const float* /*t*/, const double* F, const double* w, const int64_t* off,
                          int32_t n_events, double* wFc, double* sums, hipStream_t st) {
  if (n_events <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lc_prep, dim3(n_events), dim3(256), 0, st, F, w, off, wFc, sums);
  return hipGetLastError();
}

hipError_t launch_traj_prep_list(const double* params, int64_t n, TrajC* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_traj_prep_list, dim3((unsigned)blocks), dim3(256), 0, st, params, n, out);
  return hipGetLastError();
}

namespace {

// Scoring order of trajectory lists: each trajectory's (list, alpha bucket) key, then
// the shared bucket sort (its order holds indices over all lists).
__device__ __forceinline__ uint32_t perm_key(const TrajC* tc, int64_t i, int64_t n_traj) {
  const float a = atan2f(tc[i].sa, tc[i].ca);  // (-pi, pi]
  int b = 0;
  if (!isnan(a)) b = min(max((int)((a + 3.14159265f) * (kPermBins / 6.28318531f)), 0), kPermBins - 1);
  return (uint32_t)((i / n_traj) * kPermBins + b);
}

__global__ void k_perm_keys(const TrajC* __restrict__ tc, int64_t n, int64_t n_traj, uint32_t* key) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    key[i] = perm_key(tc, i, n_traj);
}

}  // namespace

hipError_t launch_traj_perm(const TrajC* tc, int64_t n_traj, int32_t n_lists, uint32_t* key,
                            uint32_t* hist, int32_t* perm, hipStream_t st) {
  const int64_t n = n_traj * n_lists, nb = (int64_t)n_lists * kPermBins;
  if (n <= 0) return hipSuccess;
  if (n > INT32_MAX || nb > kPermBinsMax) return hipErrorInvalidValue;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_perm_keys, dim3((unsigned)blocks), dim3(256), 0, st, tc, n, n_traj, key);
  return launch_bucket_order(key, n, (int32_t)nb, hist, perm, st);
}

hipError_t launch_traj_prep_grid(const double* axes, int32_t nu, int32_t na, int32_t nt,
                                 int32_t ne, TrajC* out, hipStream_t st) {
  const int64_t n = (int64_t)nu * na * nt * ne;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_traj_prep_grid, dim3((unsigned)blocks), dim3(256), 0, st, axes, nu, na, nt,
                     ne, out);
  return hipGetLastError();
}

hipError_t launch_search_plain(const TrajC* tc, int64_t n_traj, LcView lc, int32_t event,
                               MapC map, SearchOut out, int waves_per_block, hipStream_t st) {
  if (n_traj <= 0) return hipSuccess;
  const int threads = waves_per_block * kWave;
  int64_t blocks = (n_traj + waves_per_block - 1) / waves_per_block;
  if (blocks > 1 << 20) blocks = 1 << 20;
  hipLaunchKernelGGL(k_search_plain, dim3((unsigned)blocks), dim3(threads), 0, st, tc, n_traj, lc,
                     event, map, out);
  return hipGetLastError();
}

hipError_t launch_search_batched(const BatchedArgs& a, hipStream_t st) {
  const dim3 grid(a.grid_blocks), block(a.waves_per_block * kWave);
  switch (a.tu) {
    case 1: hipLaunchKernelGGL(k_search_batched<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_search_batched<2>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_search_batched<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_best(const double* chi2, int64_t n_seg, int64_t seg_len, double* best_chi2,
                       int64_t* best_idx, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best, dim3((unsigned)n_seg), dim3(256), 0, st, chi2, seg_len, best_chi2,
                     best_idx);
  return hipGetLastError();
}

size_t topk_scratch_bytes(int64_t n_seg, int32_t k) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(TkState) * n_seg) + al(4 * (size_t)TK_BINS * n_seg) + al(8 * (size_t)k * n_seg) +
         al(4 * (size_t)k * n_seg);
}

hipError_t launch_topk(const double* chi2, int64_t n_seg, int64_t seg_len, int32_t k,
                       double* out_chi2, int64_t* out_idx, void* scratch, int num_cu,
                       hipStream_t st) {
  if (n_seg <= 0 || k <= 0) return hipSuccess;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = (char*)scratch;
  TkState* state = (TkState*)p;
  p += al(sizeof(TkState) * n_seg);
  uint32_t* hist = (uint32_t*)p;
  p += al(4 * (size_t)TK_BINS * n_seg);
  uint64_t* keys = (uint64_t*)p;
  p += al(8 * (size_t)k * n_seg);
  uint32_t* idx = (uint32_t*)p;
  // enough workgroups to cover the chip about four times over all segments
  int64_t per_seg = (seg_len + 16 * TK_THREADS - 1) / (16 * TK_THREADS);
  const int64_t cap = std::max<int64_t>(1, (4 * (int64_t)num_cu * 4) / n_seg);
  per_seg = std::max<int64_t>(1, std::min(per_seg, cap));
  const dim3 grid((unsigned)per_seg, (unsigned)n_seg);
  hipLaunchKernelGGL(k_tk_init, dim3((unsigned)n_seg), dim3(256), 0, st, state, hist, keys, idx, n_seg,
                     seg_len, k);
  for (int pass = 0; pass < TK_PASSES; ++pass) {
    hipLaunchKernelGGL(k_tk_hist, grid, dim3(TK_THREADS), 0, st, chi2, seg_len, state, hist, pass);
    hipLaunchKernelGGL(k_tk_pick, dim3((unsigned)n_seg), dim3(TK_THREADS), 0, st, state, hist, pass);
  }
  hipLaunchKernelGGL(k_tk_collect, grid, dim3(TK_THREADS), 0, st, chi2, seg_len, k, state, keys, idx);
  hipLaunchKernelGGL(k_tk_rank, dim3((unsigned)((k + TKR_ELEMS - 1) / TKR_ELEMS), (unsigned)n_seg),
                     dim3(TKR_ELEMS * TKR_SPLIT), 0, st, chi2, seg_len, k, keys, idx, out_chi2,
                     out_idx);
  return hipGetLastError();
}

}  // namespace morse
