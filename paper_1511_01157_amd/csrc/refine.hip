// Gradient refinement of search candidates on gfx950.
//
// Chi-square gradient.  The profiled chi-square (Eqs. 5-6 of McDougall & Albrow 2015;
// sec. 4.2 bilinear map sampling) has (F_s, F_b) at their exact minimisers, so by the
// envelope theorem d chi2/d theta = -2 F_s sum w r dA/d theta with r = F - F_s A - F_b.
// One 128-lane workgroup per candidate (two wavefronts over the points, so a few
// thousand candidates still fill the chip) samples each point once and accumulates in
// FP64 the normal-equation sums with, for the directions D below, sum w D, sum w b D
// and sum w (F - Fbar) D; the fit then gives (F_s, F_b) and the sums
//   Gx = sum w r dA/dzx,  Gy = sum w r dA/dzy,
//   Gxt = sum w r tau dA/dzx,  Gyt = sum w r tau dA/dzy,
//   Ga = sum w r (zx dA/dzy - zy dA/dzx),
// from which, with zeta = tau (ca, sa) + u0 (-sa, ca) and tau = (t - t0)/tE,
//   d/dt0 = -2 F_s (-(ca Gx + sa Gy)/tE),  d/du0 = -2 F_s (-sa Gx + ca Gy),
//   d/dtE = -2 F_s (-(ca Gxt + sa Gyt)/tE), d/dalpha = -2 F_s Ga.
// dA/dzeta: on the map, k (e0 + fy (e1 - e0), ax1 - ax0) from the bilinear cell;
// off the map, A(u) = (u^2+2)/(u sqrt(u^2+4)) gives dA/du = -8/(u^2 (u^2+4)^(3/2)).
//
// L-BFGS.  One thread per candidate runs the update of the state machine (accept on the
// Armijo test or backtrack; two-loop recursion for the next direction) after the
// evaluation kernel; the state (binary32 variables p, FP64 history) is kept in
// structure-of-arrays form.  (Running the update inside the evaluation workgroup was
// slower: it raised register use and idled the workgroup during the serial update.)

#include "internal.h"

namespace morse {

namespace {

__device__ __forceinline__ double dot4(const double* a, const double* b) {
  return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3];
}

// Sum of NV FP64 values over the workgroup in a fixed order (a wavefront
// reduce-scatter, then the wave partials in wave order); every thread returns the
// same values.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*s_part)[NV]) {
  static_assert(kWave == 64 && NV <= 64, "reduce-scatter assumes 64-lane wavefronts");
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int slot = 0;
  bool valid = true;
  reduce_scatter<NV>(v, lane, slot, valid);
  if (valid) s_part[wave][slot] = v[0];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = s_part[0][q];
    for (int k = 1; k < nw; ++k) t += s_part[k][q];
    v[q] = t;
  }
  __syncthreads();
}

// One workgroup (GRAD_THREADS lanes over the points) per candidate; thread k takes the
// points k, k + GRAD_THREADS, k + 2 GRAD_THREADS, ... in increasing order.
#ifndef MORSE_GRAD_THREADS
#define MORSE_GRAD_THREADS 128
#endif
constexpr int GRAD_THREADS = MORSE_GRAD_THREADS;

struct Eval {
  double chi2, Fs, Fb;
  double g[4];
  bool valid;
};

// dA/dzeta of one sample: on the map from the bilinear cell, off the map from the
// point-source magnification.
__device__ __forceinline__ void sample_dA(const Sample& sm, double kx, double ky, double& dAx,
                                          double& dAy) {
  if (sm.on) {
    const double e0 = (double)sm.e0, e1 = (double)sm.e1;
    dAx = kx * (e0 + (double)sm.fy * (e1 - e0));
    dAy = ky * ((double)sm.ax1 - (double)sm.ax0);
  } else {
    // dA/dzeta = dA/du zeta/u = -8 zeta / (u^2 (u^2+4) sqrt(u^2 (u^2+4)))
    const double zx = (double)sm.zx, zy = (double)sm.zy;
    const double u2 = zx * zx + zy * zy;
    const double pp = u2 * (u2 + 4.0);
    const double f = -8.0 / (pp * sqrt(pp));
    dAx = f * zx;
    dAy = f * zy;
  }
}

// Number of derivative directions D (dA/dzx, dA/dzy, tau dA/dzx, tau dA/dzy,
// zx dA/dzy - zy dA/dzx) and of one-pass sums (3 fit sums + 3 per direction).
constexpr int kDirs = 5;
constexpr int kSums = 3 + 3 * kDirs;

// chi2, (F_s, F_b) and the gradient of candidate c (every thread returns the same).
// With an anchor the parameters are the L-BFGS variables and the gradient is with
// respect to them.
//
// One pass: with b = A - 1, wFc = w (F - Fbar) and c0 = B1/S_w the residual is
// r = (F - Fbar) - F_s (b - c0), so for every direction D
//   sum w r D = P_D - F_s (Q_D - c0 R_D),  P_D = sum wFc D, Q_D = sum w b D, R_D = sum w D,
// and chi2 = V - F_s C (the search's one-pass fit).  When the fit is degenerate or that
// chi2 is flagged as cancellation-prone, a second pass sums w r^2 and w r D directly
// with the residual formed point by point.
__device__ Eval grad_eval(const GradArgs& a, int64_t c, double (*s_part)[kSums]) {
  Eval out;
  const int tid = threadIdx.x;
  const int32_t e = uniform(a.event[c]);
  const int32_t mi = uniform(a.mapidx[c]);
  out.valid = !(e < 0 || e >= a.n_events || mi < 0 || mi >= a.n_maps);
  if (!out.valid) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    out.chi2 = out.Fs = out.Fb = nan;
    for (int q = 0; q < 4; ++q) out.g[q] = nan;
    return out;
  }
  const MapC m = uniform(a.maps[mi]);
  const TrajC tc = uniform(a.tc[c]);
  const double tE = uniform(a.tEv[c]);
  const double tE_anchor = a.anchor ? uniform(a.anchor[4 * c + 2]) : 0.0;
  const float iE = tc.iE, ca = tc.ca, sa = tc.sa, bx = tc.bx, by = tc.by;
  const float t0p = (float)(tc.t0 - uniform(a.lc.t_ref[e]));

  const int64_t p0 = uniform(a.lc.off[e]);
  const int32_t np = (int32_t)(uniform(a.lc.off[e + 1]) - p0);
  const float* t = a.lc.t + p0;
  const double* w = a.lc.w + p0;
  const double* wFc = a.lc.wFc + p0;
  const double* F = a.lc.F + p0;
  const double Sw = uniform(a.lc.sums[3 * e]), Fbar = uniform(a.lc.sums[3 * e + 1]),
               V = uniform(a.lc.sums[3 * e + 2]);
  const double kx = (double)m.kx, ky = (double)m.ky;

  // acc: B1, B2, C, then (R_D, Q_D, P_D) per direction
  double acc[kSums];
#pragma unroll
  for (int q = 0; q < kSums; ++q) acc[q] = 0.0;
  // The point at time tl: tau and the source position are recomputed from tl (the
  // same operations as locate, so the same bits) rather than kept live across the
  // gathers, which keeps the kernel within 96 VGPRs: five wavefronts per SIMD.
  auto add_point = [&](const Loc& l, float tl, const Quad& v, double wi, double wfc) {
    float tr = tl;
    asm volatile("" : "+v"(tr));  // opaque copy: the compiler cannot reuse locate's values
    const float ltau = (tr - t0p) * iE;
    const float lzx = ltau * ca + bx, lzy = ltau * sa + by;
    const float e0 = v.v10 - v.v00, e1 = v.v11 - v.v01;
    const float ax0 = v.v00 + l.fx * e0, ax1 = v.v01 + l.fx * e1;
    float A = ax0 + l.fy * (ax1 - ax0);
    double dAx = kx * ((double)e0 + (double)l.fy * ((double)e1 - (double)e0));
    double dAy = ky * ((double)ax1 - (double)ax0);
    if (!l.on) {
      A = point_lens_A(lzx, lzy);
      // dA/dzeta = dA/du zeta/u = -8 zeta / (u^2 (u^2+4) sqrt(u^2 (u^2+4)))
      const double zx = (double)lzx, zy = (double)lzy;
      const double u2 = zx * zx + zy * zy;
      const double pp = u2 * (u2 + 4.0);
      const double f = -8.0 / (pp * sqrt(pp));
      dAx = f * zx;
      dAy = f * zy;
    }
    const double b = (double)A - 1.0;
    const double wb = wi * b;
    acc[0] += wb;
    acc[1] = fma(wb, b, acc[1]);
    acc[2] = fma(b, wfc, acc[2]);
    const double tau = (double)ltau;
    const double D[kDirs] = {dAx, dAy, dAx * tau, dAy * tau,
                             (double)lzx * dAy - (double)lzy * dAx};
#pragma unroll
    for (int k = 0; k < kDirs; ++k) {
      acc[3 + 3 * k] = fma(wi, D[k], acc[3 + 3 * k]);
      acc[4 + 3 * k] = fma(wb, D[k], acc[4 + 3 * k]);
      acc[5 + 3 * k] = fma(wfc, D[k], acc[5 + 3 * k]);
    }
  };
  // Software pipeline over two register sets (a, b), so that nothing is copied between
  // iterations: while one point is added, the cell and weights of the next point and
  // the time of the one after are in flight.  Loads past the end are clamped to the
  // last point and never added.
  constexpr int32_t STEP = GRAD_THREADS;
  auto idx = [&](int32_t j) -> uint32_t { return (uint32_t)(j < np ? j : np - 1); };
  float tla = ldg(t, idx(tid));
  Loc la = locate(m, tla, t0p, iE, ca, sa, bx, by);
  Quad va = ldq(m, la.q);
  double wa = ldg(w, idx(tid)), fa = ldg(wFc, idx(tid));
  float ta = ldg(t, idx(tid + STEP));
  for (int32_t i0 = tid; i0 < np; i0 += 2 * STEP) {
    // set b: point i0 + STEP (time ta); time of i0 + 2 STEP
    const float tb = ldg(t, idx(i0 + 2 * STEP));
    const float tlb = ta;
    const Loc lb = locate(m, ta, t0p, iE, ca, sa, bx, by);
    const Quad vb = ldq(m, lb.q);
    const double wb = ldg(w, idx(i0 + STEP)), fb = ldg(wFc, idx(i0 + STEP));
    add_point(la, tla, va, wa, fa);
    // set a: point i0 + 2 STEP (time tb); time of i0 + 3 STEP
    ta = ldg(t, idx(i0 + 3 * STEP));
    tla = tb;
    la = locate(m, tb, t0p, iE, ca, sa, bx, by);
    va = ldq(m, la.q);
    wa = ldg(w, idx(i0 + 2 * STEP));
    fa = ldg(wFc, idx(i0 + 2 * STEP));
    if (i0 + STEP < np) add_point(lb, tlb, vb, wb, fb);
  }
  block_sum<kSums>(acc, s_part);
  const Fit fit = centred_fit(Sw, Fbar, V, acc[0], acc[1], acc[2], fit_terms(np, GRAD_THREADS));
  const double Fs = fit.Fs, Fb = fit.Fb;
  double G[kDirs];  // sum w r D
  double chi2;
  if (!fit.degenerate && !fit.recheck) {
    const double c0 = acc[0] / Sw;
#pragma unroll
    for (int k = 0; k < kDirs; ++k)
      G[k] = acc[5 + 3 * k] - Fs * (acc[4 + 3 * k] - c0 * acc[3 + 3 * k]);
    chi2 = fit.chi2;
  } else {  // uniform per workgroup: the sums are identical on every thread
    // direct sums of w r^2 and w r D, Neumaier-compensated per thread
    double n2[1 + kDirs], n2c[1 + kDirs];
#pragma unroll
    for (int q = 0; q <= kDirs; ++q) n2[q] = n2c[q] = 0.0;
    for (int32_t i = tid; i < np; i += GRAD_THREADS) {
      const uint32_t u = (uint32_t)i;
      const Sample sm = sample_full(m, ldg(t, u), t0p, iE, ca, sa, bx, by);
      const double A = (double)sm.A;
      const double r = ldg(F, u) - Fs * A - Fb;
      const double wr = ldg(w, u) * r;
      double dAx, dAy;
      sample_dA(sm, kx, ky, dAx, dAy);
      const double tau = (double)sm.tau;
      neumaier_add(n2[0], n2c[0], wr * r);
      neumaier_add(n2[1], n2c[1], wr * dAx);
      neumaier_add(n2[2], n2c[2], wr * dAy);
      neumaier_add(n2[3], n2c[3], (wr * dAx) * tau);
      neumaier_add(n2[4], n2c[4], (wr * dAy) * tau);
      neumaier_add(n2[5], n2c[5], wr * ((double)sm.zx * dAy - (double)sm.zy * dAx));
    }
#pragma unroll
    for (int q = 0; q <= kDirs; ++q) n2[q] += n2c[q];
    // reuse the first 1 + kDirs columns of the partial-sum buffer
    block_sum<1 + kDirs>(n2, reinterpret_cast<double (*)[1 + kDirs]>(&s_part[0][0]));
    chi2 = n2[0];
#pragma unroll
    for (int k = 0; k < kDirs; ++k) G[k] = n2[1 + k];
  }
  const double c64 = (double)ca, s64 = (double)sa;
  const double k2 = -2.0 * Fs;
  out.g[0] = k2 * (-(c64 * G[0] + s64 * G[1]) / tE);
  out.g[1] = k2 * (-s64 * G[0] + c64 * G[1]);
  out.g[2] = k2 * (-(c64 * G[2] + s64 * G[3]) / tE);
  out.g[3] = k2 * G[4];
  if (a.anchor) {  // gradient with respect to the scaled variables
    out.g[0] = out.g[0] * tE_anchor;
    out.g[2] = out.g[2] * tE;
  }
  out.chi2 = chi2;
  out.Fs = Fs;
  out.Fb = Fb;
  return out;
}

// Trajectory constants of natural parameters (t0, u0, tE, alpha), FP64 trigonometry
// rounded once, written for candidate c.
__device__ void write_natural(const GradArgs& a, int64_t c, double t0, double u0, double tE,
                              double al) {
  double sn, cs;
  sincos(al, &sn, &cs);
  TrajC r;
  r.t0 = t0;
  r.iE = (float)(1.0 / tE);
  r.ca = (float)cs;
  r.sa = (float)sn;
  r.bx = (float)(-u0 * sn);
  r.by = (float)(u0 * cs);
  r.pad = 0.0f;
  a.tc[c] = r;
  a.tEv[c] = tE;
}

// Natural parameters from the L-BFGS anchor and binary32 displacement p.
__device__ void write_traj(const GradArgs& a, int64_t c, const double* an, const float* p) {
  write_natural(a, c, an[0] + (double)p[0] * an[2], an[1] + (double)p[1],
                an[2] * exp((double)p[2]), an[3] + (double)p[3]);
}

// Candidate c's trajectory constants: from its FP64 row, or from its anchor and trial
// displacement.
__device__ void prep_candidate(const GradArgs& a, int64_t c) {
  if (a.anchor) {
    write_traj(a, c, a.anchor + 4 * c, a.pt + 4 * c);
  } else {
    const double* p = a.params + 4 * c;
    write_natural(a, c, p[0], p[1], p[2], p[3]);
  }
}

__global__ void k_cand_prep(GradArgs a) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  if (a.active && !a.active[c]) return;
  prep_candidate(a, c);
}

// Workgroups are dispatched to the 8 XCDs in turn (the grid is a multiple of 8), so
// slot s runs on XCD s % 8.  With an evaluation order grouped by map, slot s takes the
// s-th candidate of that order: the XCDs work through the same map at the same time
// and share it in the last-level cache.  Without one, XCD x takes the contiguous
// candidate range [x per, (x + 1) per), so that neighbouring candidates (similar
// trajectories after a ranked selection) share its L2.
// At most 96 VGPRs (five wavefronts per SIMD): the compiler fits the kernel without
// spilling (four wavefronts measured 2% slower).
__global__ __launch_bounds__(GRAD_THREADS) __attribute__((amdgpu_waves_per_eu(5))) void k_chi2_grad(GradArgs a) {
  __shared__ double s_part[GRAD_THREADS / kWave][kSums];
  const int64_t per = (a.n + 7) / 8;
  for (int64_t slot = blockIdx.x; slot < 8 * per; slot += gridDim.x) {
    const int64_t pos = a.order ? slot : (slot % 8) * per + slot / 8;
    if (pos >= a.n) continue;
    const int64_t c = a.order ? (int64_t)uniform(a.order[pos]) : pos;
    if (a.active && !a.active[c]) continue;  // uniform per workgroup
    const Eval ev = grad_eval(a, c, s_part);
    if (threadIdx.x == 0) {
      if (a.chi2) a.chi2[c] = ev.chi2;
      if (a.grad)
        for (int q = 0; q < 4; ++q) a.grad[4 * c + q] = ev.g[q];
      if (a.fs) a.fs[c] = ev.Fs;
      if (a.fb) a.fb[c] = ev.Fb;
    }
  }
}

// One candidate's L-BFGS state, held in registers for one update.  The history pairs
// are stored oldest first (an accepted pair past m shifts the others down), so all of
// them, like every other field, load at once at the start of the update, with no load
// waiting on another or on a store.  M >= m bounds the history; loops run over
// compile-time slots in the order of a loop over the nh stored pairs.
template <int M>
struct Regs {
  double S[M][4], Y[M][4], R[M];
  double g[4], d[4], f, step;
  float p[4], pt[4];
  int nh, nls;
};

template <int M>
__device__ __forceinline__ void load_regs(const LbfgsState& s, int64_t c, Regs<M>& q) {
#pragma unroll
  for (int h = 0; h < M; ++h) {  // slots past nh hold stale values and are never used
    const int64_t row = c * s.m + min(h, s.m - 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q.S[h][k] = s.S[row * 4 + k];
      q.Y[h][k] = s.Y[row * 4 + k];
    }
    q.R[h] = s.R[row];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    q.g[k] = s.g[4 * c + k];
    q.d[k] = s.d[4 * c + k];
    q.p[k] = s.p[4 * c + k];
    q.pt[k] = s.pt[4 * c + k];
  }
  q.f = s.f[c];
  q.step = s.step[c];
  q.nh = s.nhist[c];
  q.nls = s.nls[c];
}

// New search direction at the accepted point (q.p, q.g); stores d, step, nls, pt and
// may stop the candidate when the trial would not move it.  Returns whether it moved.
template <int M>
__device__ bool new_direction(const LbfgsState& s, int64_t c, Regs<M>& q) {
  const int nh = q.nh;
  double r[4], d[4], qq[4], alph[M];
  for (int k = 0; k < 4; ++k) qq[k] = q.g[k];
#pragma unroll
  for (int h = M - 1; h >= 0; --h) {
    if (h < nh) {
      const double a = q.R[h] * dot4(q.S[h], qq);
      alph[h] = a;
      for (int k = 0; k < 4; ++k) qq[k] = qq[k] - a * q.Y[h][k];
    }
  }
  const double gn = sqrt(dot4(q.g, q.g));
  double gamma = gn > 0.0 ? 1e-2 / gn : 0.0;
#pragma unroll
  for (int h = 0; h < M; ++h)
    if (h == nh - 1) gamma = dot4(q.S[h], q.Y[h]) / dot4(q.Y[h], q.Y[h]);
  for (int k = 0; k < 4; ++k) r[k] = gamma * qq[k];
#pragma unroll
  for (int h = 0; h < M; ++h) {
    if (h < nh) {
      const double b = q.R[h] * dot4(q.Y[h], r);
      for (int k = 0; k < 4; ++k) r[k] = r[k] + q.S[h][k] * (alph[h] - b);
    }
  }
  for (int k = 0; k < 4; ++k) d[k] = -r[k];
  const double gd = dot4(q.g, d);
  bool finite = true;
  for (int k = 0; k < 4; ++k) finite = finite && isfinite(d[k]);
  if (!(gd < 0.0) || !finite) {
    q.nh = 0;
    s.nhist[c] = 0;
    gamma = gn > 0.0 ? 1e-2 / gn : 0.0;
    for (int k = 0; k < 4; ++k) d[k] = -(gamma * q.g[k]);
  }
  s.step[c] = 1.0;
  s.nls[c] = 0;
  bool moved = false;
  for (int k = 0; k < 4; ++k) {
    s.d[4 * c + k] = d[k];
    const float v = (float)((double)q.p[k] + 1.0 * d[k]);
    q.pt[k] = v;
    s.pt[4 * c + k] = v;
    moved = moved || (v != q.p[k]);
  }
  if (!moved) s.active[c] = 0;
  return moved;
}

// One update of the state machine for candidate c given the evaluation (ft, gt) at
// its trial point; returns whether the candidate is still active (its next trial
// point is then q.pt).
template <int M>
__device__ bool lbfgs_step(const LbfgsState& s, int64_t c, int32_t round, double ft,
                           const double* gt, Regs<M>& q) {
  if (round == 0) {
    for (int k = 0; k < 4; ++k) {
      q.p[k] = q.pt[k];
      q.g[k] = gt[k];
      s.p[4 * c + k] = q.p[k];
      s.g[4 * c + k] = q.g[k];
    }
    q.f = ft;
    s.f[c] = ft;
    q.nh = 0;
    return new_direction<M>(s, c, q);
  }
  const double gd = dot4(q.g, q.d);
  const double t = q.step;
  if (isfinite(ft) && ft <= q.f + (s.c1 * t) * gd) {
    double sv[4], yv[4];
    for (int k = 0; k < 4; ++k) {
      sv[k] = (double)q.pt[k] - (double)q.p[k];
      yv[k] = gt[k] - q.g[k];
    }
    const double sy = dot4(sv, yv);
    if (sy > 1e-12 * sqrt(dot4(sv, sv)) * sqrt(dot4(yv, yv))) {
      const double rho = 1.0 / sy;
      const int m = s.m;
      if (q.nh == m) {  // full: drop the oldest pair
#pragma unroll
        for (int h = 0; h + 1 < M; ++h)
          if (h + 1 < m) {
            for (int k = 0; k < 4; ++k) {
              q.S[h][k] = q.S[h + 1][k];
              q.Y[h][k] = q.Y[h + 1][k];
            }
            q.R[h] = q.R[h + 1];
          }
        q.nh = m - 1;
      }
#pragma unroll
      for (int h = 0; h < M; ++h)
        if (h == q.nh) {
          for (int k = 0; k < 4; ++k) {
            q.S[h][k] = sv[k];
            q.Y[h][k] = yv[k];
          }
          q.R[h] = rho;
        }
      q.nh += 1;
#pragma unroll
      for (int h = 0; h < M; ++h)  // write the history back, oldest first
        if (h < q.nh) {
          const int64_t row = c * s.m + h;
          for (int k = 0; k < 4; ++k) {
            s.S[row * 4 + k] = q.S[h][k];
            s.Y[row * 4 + k] = q.Y[h][k];
          }
          s.R[row] = q.R[h];
        }
      s.nhist[c] = q.nh;
    }
    for (int k = 0; k < 4; ++k) {
      q.p[k] = q.pt[k];
      q.g[k] = gt[k];
      s.p[4 * c + k] = q.p[k];
      s.g[4 * c + k] = q.g[k];
    }
    q.f = ft;
    s.f[c] = ft;
    return new_direction<M>(s, c, q);
  }
  const int n = q.nls + 1;
  s.nls[c] = n;
  if (n >= s.max_ls) {
    s.active[c] = 0;
    return false;
  }
  const double tn = t * s.shrink;
  s.step[c] = tn;
  for (int k = 0; k < 4; ++k) {
    q.pt[k] = (float)((double)q.p[k] + tn * q.d[k]);
    s.pt[4 * c + k] = q.pt[k];
  }
  return true;
}

// Start of a refinement: anchor = the candidate's row, p_t = 0, empty history, every
// candidate active, and the trajectory constants of the first trial point.
__global__ void k_refine_init(LbfgsState s, GradArgs a, const double* params,
                              double* anchor) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= s.n) return;
  for (int k = 0; k < 4; ++k) {
    anchor[4 * c + k] = params[4 * c + k];
    s.pt[4 * c + k] = 0.0f;
  }
  s.nhist[c] = 0;
  s.nls[c] = 0;
  s.active[c] = 1;
  prep_candidate(a, c);
}

// Update of every active candidate from its evaluation (ft, gt), then the trajectory
// constants of its next trial point; round 0 also records the starting chi-square.
template <int M>
__global__ __launch_bounds__(64) void k_lbfgs_update(LbfgsState s, GradArgs a, int32_t round,
                               const double* __restrict__ ft, const double* __restrict__ gt,
                               double* __restrict__ chi2_init) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= s.n || !s.active[c]) return;
  double g[4], an[4];
  for (int k = 0; k < 4; ++k) {
    g[k] = gt[4 * c + k];
    an[k] = s.anchor[4 * c + k];
  }
  const double f = ft[c];
  Regs<M> q;
  load_regs<M>(s, c, q);
  if (round == 0 && chi2_init) chi2_init[c] = f;
  if (lbfgs_step<M>(s, c, round, f, g, q)) write_traj(a, c, an, q.pt);
}

__global__ void k_lbfgs_finish(LbfgsState s, double* params, double* chi2_out) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= s.n) return;
  const double* an = s.anchor + 4 * c;
  const float* p = s.p + 4 * c;
  params[4 * c + 0] = an[0] + (double)p[0] * an[2];
  params[4 * c + 1] = an[1] + (double)p[1];
  params[4 * c + 2] = an[2] * exp((double)p[2]);
  params[4 * c + 3] = an[3] + (double)p[3];
  if (chi2_out) chi2_out[c] = s.f[c];
}

}  // namespace

hipError_t launch_cand_prep(const GradArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cand_prep, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

namespace {

// Evaluation order: each candidate's (map, event) key, then the shared bucket sort.
__device__ __forceinline__ uint32_t order_key(const GradArgs& a, int64_t c, bool by_event) {
  const int32_t e = a.event[c], m = a.mapidx[c];
  if (e < 0 || e >= a.n_events || m < 0 || m >= a.n_maps) return 0u;  // NaN outputs anyway
  return by_event ? (uint32_t)m * (uint32_t)a.n_events + (uint32_t)e : (uint32_t)m;
}

__global__ void k_order_keys(GradArgs a, bool by_event, uint32_t* key) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.n;
       c += (int64_t)gridDim.x * blockDim.x)
    key[c] = order_key(a, c, by_event);
}

}  // namespace

hipError_t launch_cand_order(const GradArgs& a, uint32_t* key, uint32_t* hist, int32_t* order,
                             hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n > INT32_MAX || a.n_maps <= 0 || a.n_events <= 0) return hipErrorInvalidValue;
  const int64_t nb = order_bins(a.n_maps, a.n_events);
  const bool by_event = nb == (int64_t)a.n_maps * a.n_events;
  int64_t blocks = (a.n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_order_keys, dim3((unsigned)blocks), dim3(256), 0, st, a, by_event, key);
  return launch_bucket_order(key, a.n, (int32_t)nb, hist, order, st);
}

hipError_t launch_chi2_grad(const GradArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  int64_t blocks = 8 * ((a.n + 7) / 8);
  if (blocks > 1 << 20) blocks = 1 << 20;
  hipLaunchKernelGGL(k_chi2_grad, dim3((unsigned)blocks), dim3(GRAD_THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_refine_init(const LbfgsState& s, const GradArgs& a, const double* params,
                              double* anchor, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_init, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, s, a,
                     params, anchor);
  return hipGetLastError();
}

hipError_t launch_lbfgs_update(const LbfgsState& s, const GradArgs& a, int32_t round,
                               const double* ft, const double* gt, double* chi2_init,
                               hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  // 64-lane workgroups: one thread per candidate, spread over as many CUs as possible
  const dim3 grid((unsigned)((s.n + 63) / 64)), block(64);
  if (s.m <= 8)
    hipLaunchKernelGGL(k_lbfgs_update<8>, grid, block, 0, st, s, a, round, ft, gt, chi2_init);
  else
    hipLaunchKernelGGL(k_lbfgs_update<16>, grid, block, 0, st, s, a, round, ft, gt, chi2_init);
  return hipGetLastError();
}

hipError_t launch_lbfgs_finish(const LbfgsState& s, double* params, double* chi2_out,
                               hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbfgs_finish, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, s,
                     params, chi2_out);
  return hipGetLastError();
}

}  // namespace morse
