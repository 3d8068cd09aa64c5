// Gradient refinement of search candidates on gfx950.
//
// Chi-square gradient.  The profiled chi-square (Eqs. 5-6 of McDougall & Albrow 2015;
// sec. 4.2 bilinear map sampling) has (F_s, F_b) at their exact minimisers, so by the
// envelope theorem d chi2/d theta = -2 F_s sum w r dA/d theta with r = F - F_s A - F_b.
// One 256-lane workgroup per candidate (four wavefronts over the points, so a few
// thousand candidates still fill the chip): pass 1 accumulates the normal-equation
// sums and solves for (F_s, F_b) as the search does; pass 2 re-samples each point,
// forms r, and accumulates in FP64
//   chi2 = sum w r^2,  Gx = sum w r dA/dzx,  Gy = sum w r dA/dzy,
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

// Sum of one FP64 value over the workgroup in a fixed order (wave butterflies, then
// the wave partials in wave order); every thread returns the same value.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*s_part)[NV]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) s_part[wave][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = s_part[0][q];
    for (int k = 1; k < nw; ++k) t += s_part[k][q];
    v[q] = t;
  }
  __syncthreads();
}

// One workgroup (GRAD_THREADS lanes over the points) per candidate.
constexpr int GRAD_THREADS = 256;

struct Eval {
  double chi2, Fs, Fb;
  double g[4];
  bool valid;
};

// chi2, (F_s, F_b) and the gradient of candidate c (every thread returns the same).
// With an anchor the parameters are the L-BFGS variables and the gradient is with
// respect to them.
__device__ Eval grad_eval(const GradArgs& a, int64_t c, double (*s3)[3], double (*s6)[6]) {
  Eval out;
  const int tid = threadIdx.x;
  const int32_t e = a.event[c];
  const int32_t mi = a.mapidx[c];
  out.valid = !(e < 0 || e >= a.n_events || mi < 0 || mi >= a.n_maps);
  if (!out.valid) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    out.chi2 = out.Fs = out.Fb = nan;
    for (int q = 0; q < 4; ++q) out.g[q] = nan;
    return out;
  }
  const MapC m = a.maps[mi];
  const TrajC tc = a.tc[c];
  const double tE = a.tEv[c];
  const double tE_anchor = a.anchor ? a.anchor[4 * c + 2] : 0.0;
  const float iE = tc.iE, ca = tc.ca, sa = tc.sa, bx = tc.bx, by = tc.by;
  const float t0p = (float)(tc.t0 - a.lc.t_ref[e]);

  const int64_t p0 = a.lc.off[e];
  const int32_t np = (int32_t)(a.lc.off[e + 1] - p0);
  const float* t = a.lc.t + p0;
  const double* w = a.lc.w + p0;
  const double* wFc = a.lc.wFc + p0;
  const double* F = a.lc.F + p0;
  const double Sw = a.lc.sums[3 * e], Fbar = a.lc.sums[3 * e + 1], V = a.lc.sums[3 * e + 2];

  // pass 1: normal-equation sums (centred form) and the profiled fit
  double n1[3] = {0.0, 0.0, 0.0};
  for (int32_t i = tid; i < np; i += GRAD_THREADS) {
    const uint32_t u = (uint32_t)i;
    const double b = (double)sample_A(m, ldg(t, u), t0p, iE, ca, sa, bx, by) - 1.0;
    const double wb = ldg(w, u) * b;
    n1[0] += wb;
    n1[1] = fma(wb, b, n1[1]);
    n1[2] = fma(b, ldg(wFc, u), n1[2]);
  }
  block_sum<3>(n1, s3);
  const Fit fit = centred_fit(Sw, Fbar, V, n1[0], n1[1], n1[2]);
  const double Fs = fit.Fs, Fb = fit.Fb;

  // pass 2: residuals, direct chi-square and gradient sums
  const double kx = (double)m.kx, ky = (double)m.ky;
  double n2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // chi, Gx, Gy, Gxt, Gyt, Ga
  for (int32_t i = tid; i < np; i += GRAD_THREADS) {
    const uint32_t u = (uint32_t)i;
    const Sample sm = sample_full(m, ldg(t, u), t0p, iE, ca, sa, bx, by);
    const double A = (double)sm.A;
    const double r = ldg(F, u) - Fs * A - Fb;
    const double wr = ldg(w, u) * r;
    const double zx = (double)sm.zx, zy = (double)sm.zy, tau = (double)sm.tau;
    double dAx, dAy;
    if (sm.on) {
      const double e0 = (double)sm.e0, e1 = (double)sm.e1;
      dAx = kx * (e0 + (double)sm.fy * (e1 - e0));
      dAy = ky * ((double)sm.ax1 - (double)sm.ax0);
    } else {
      // dA/dzeta = dA/du zeta/u = -8 zeta / (u^2 (u^2+4) sqrt(u^2 (u^2+4)))
      const double u2 = zx * zx + zy * zy;
      const double pp = u2 * (u2 + 4.0);
      const double f = -8.0 / (pp * sqrt(pp));
      dAx = f * zx;
      dAy = f * zy;
    }
    n2[0] = fma(wr, r, n2[0]);
    n2[1] = fma(wr, dAx, n2[1]);
    n2[2] = fma(wr, dAy, n2[2]);
    n2[3] = fma(wr * dAx, tau, n2[3]);
    n2[4] = fma(wr * dAy, tau, n2[4]);
    n2[5] = fma(wr, zx * dAy - zy * dAx, n2[5]);
  }
  block_sum<6>(n2, s6);
  const double c64 = (double)ca, s64 = (double)sa;
  const double k2 = -2.0 * Fs;
  out.g[0] = k2 * (-(c64 * n2[1] + s64 * n2[2]) / tE);
  out.g[1] = k2 * (-s64 * n2[1] + c64 * n2[2]);
  out.g[2] = k2 * (-(c64 * n2[3] + s64 * n2[4]) / tE);
  out.g[3] = k2 * n2[5];
  if (a.anchor) {  // gradient with respect to the scaled variables
    out.g[0] = out.g[0] * tE_anchor;
    out.g[2] = out.g[2] * tE;
  }
  out.chi2 = n2[0];
  out.Fs = Fs;
  out.Fb = Fb;
  return out;
}

// Natural parameters of each candidate (from the FP64 rows, or from the L-BFGS anchor
// and binary32 displacement) -> trajectory constants, FP64 trigonometry rounded once.
__global__ void k_cand_prep(GradArgs a) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  if (a.active && !a.active[c]) return;
  double t0, u0, tE, al;
  if (a.anchor) {
    const double* an = a.anchor + 4 * c;
    const float* p = a.pt + 4 * c;
    t0 = an[0] + (double)p[0] * an[2];
    u0 = an[1] + (double)p[1];
    tE = an[2] * exp((double)p[2]);
    al = an[3] + (double)p[3];
  } else {
    const double* p = a.params + 4 * c;
    t0 = p[0];
    u0 = p[1];
    tE = p[2];
    al = p[3];
  }
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

__global__ __launch_bounds__(GRAD_THREADS) void k_chi2_grad(GradArgs a) {
  __shared__ double s3[GRAD_THREADS / kWave][3];
  __shared__ double s6[GRAD_THREADS / kWave][6];
  for (int64_t c = blockIdx.x; c < a.n; c += gridDim.x) {
    if (a.active && !a.active[c]) continue;  // uniform per workgroup
    const Eval ev = grad_eval(a, c, s3, s6);
    if (threadIdx.x == 0) {
      if (a.chi2) a.chi2[c] = ev.chi2;
      if (a.grad)
        for (int q = 0; q < 4; ++q) a.grad[4 * c + q] = ev.g[q];
      if (a.fs) a.fs[c] = ev.Fs;
      if (a.fb) a.fb[c] = ev.Fb;
    }
  }
}

constexpr int kMaxHist = 16;

struct Cand {
  const LbfgsState& s;
  int64_t c;
  __device__ double* S(int slot) const { return s.S + ((c * s.m + slot) * 4); }
  __device__ double* Y(int slot) const { return s.Y + ((c * s.m + slot) * 4); }
};

// New search direction at the accepted point (p, g); sets d, step, nls, pt and may
// stop the candidate when the trial would not move it.
__device__ void new_direction(const LbfgsState& s, int64_t c) {
  Cand cd{s, c};
  double g[4], q[4], r[4], d[4], alph[kMaxHist];
  for (int k = 0; k < 4; ++k) g[k] = s.g[4 * c + k];
  int nh = s.nhist[c];
  int st = s.start[c];
  for (int k = 0; k < 4; ++k) q[k] = g[k];
  for (int h = nh - 1; h >= 0; --h) {
    const int slot = (st + h) % s.m;
    const double a = s.R[c * s.m + slot] * dot4(cd.S(slot), q);
    alph[h] = a;
    for (int k = 0; k < 4; ++k) q[k] = q[k] - a * cd.Y(slot)[k];
  }
  const double gn = sqrt(dot4(g, g));
  double gamma;
  if (nh > 0) {
    const int slot = (st + nh - 1) % s.m;
    gamma = dot4(cd.S(slot), cd.Y(slot)) / dot4(cd.Y(slot), cd.Y(slot));
  } else {
    gamma = gn > 0.0 ? 1e-2 / gn : 0.0;
  }
  for (int k = 0; k < 4; ++k) r[k] = gamma * q[k];
  for (int h = 0; h < nh; ++h) {
    const int slot = (st + h) % s.m;
    const double b = s.R[c * s.m + slot] * dot4(cd.Y(slot), r);
    for (int k = 0; k < 4; ++k) r[k] = r[k] + cd.S(slot)[k] * (alph[h] - b);
  }
  for (int k = 0; k < 4; ++k) d[k] = -r[k];
  const double gd = dot4(g, d);
  bool finite = true;
  for (int k = 0; k < 4; ++k) finite = finite && isfinite(d[k]);
  if (!(gd < 0.0) || !finite) {
    s.nhist[c] = 0;
    s.start[c] = 0;
    gamma = gn > 0.0 ? 1e-2 / gn : 0.0;
    for (int k = 0; k < 4; ++k) d[k] = -(gamma * g[k]);
  }
  s.step[c] = 1.0;
  s.nls[c] = 0;
  bool moved = false;
  for (int k = 0; k < 4; ++k) {
    s.d[4 * c + k] = d[k];
    const float pk = s.p[4 * c + k];
    const float v = (float)((double)pk + 1.0 * d[k]);
    s.pt[4 * c + k] = v;
    moved = moved || (v != pk);
  }
  if (!moved) s.active[c] = 0;
}

// One update of the state machine for candidate c given the evaluation (ft, gt) at
// its trial point.
__device__ void lbfgs_step(const LbfgsState& s, int64_t c, int32_t round, double ft,
                           const double* gt) {
  if (round == 0) {
    for (int k = 0; k < 4; ++k) {
      s.p[4 * c + k] = s.pt[4 * c + k];
      s.g[4 * c + k] = gt[k];
    }
    s.f[c] = ft;
    new_direction(s, c);
    return;
  }
  double g[4], d[4];
  for (int k = 0; k < 4; ++k) {
    g[k] = s.g[4 * c + k];
    d[k] = s.d[4 * c + k];
  }
  const double gd = dot4(g, d);
  const double t = s.step[c];
  if (isfinite(ft) && ft <= s.f[c] + (s.c1 * t) * gd) {
    double sv[4], yv[4];
    for (int k = 0; k < 4; ++k) {
      sv[k] = (double)s.pt[4 * c + k] - (double)s.p[4 * c + k];
      yv[k] = gt[k] - g[k];
    }
    const double sy = dot4(sv, yv);
    if (sy > 1e-12 * sqrt(dot4(sv, sv)) * sqrt(dot4(yv, yv))) {
      const int nh = s.nhist[c];
      const int st = s.start[c];
      int slot;
      if (nh < s.m) {
        slot = (st + nh) % s.m;
        s.nhist[c] = nh + 1;
      } else {
        slot = st;
        s.start[c] = (st + 1) % s.m;
      }
      Cand cd{s, c};
      for (int k = 0; k < 4; ++k) {
        cd.S(slot)[k] = sv[k];
        cd.Y(slot)[k] = yv[k];
      }
      s.R[c * s.m + slot] = 1.0 / sy;
    }
    for (int k = 0; k < 4; ++k) {
      s.p[4 * c + k] = s.pt[4 * c + k];
      s.g[4 * c + k] = gt[k];
    }
    s.f[c] = ft;
    new_direction(s, c);
  } else {
    const int n = s.nls[c] + 1;
    s.nls[c] = n;
    if (n >= s.max_ls) {
      s.active[c] = 0;
    } else {
      const double tn = t * s.shrink;
      s.step[c] = tn;
      for (int k = 0; k < 4; ++k)
        s.pt[4 * c + k] = (float)((double)s.p[4 * c + k] + tn * d[k]);
    }
  }
}

__global__ void k_lbfgs_update(LbfgsState s, int32_t round, const double* __restrict__ ft,
                               const double* __restrict__ gt) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= s.n || !s.active[c]) return;
  double g[4];
  for (int k = 0; k < 4; ++k) g[k] = gt[4 * c + k];
  lbfgs_step(s, c, round, ft[c], g);
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

hipError_t launch_chi2_grad(const GradArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  int64_t blocks = a.n;
  if (blocks > 1 << 20) blocks = 1 << 20;
  hipLaunchKernelGGL(k_chi2_grad, dim3((unsigned)blocks), dim3(GRAD_THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_lbfgs_update(const LbfgsState& s, int32_t round, const double* ft,
                               const double* gt, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbfgs_update, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, s,
                     round, ft, gt);
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
