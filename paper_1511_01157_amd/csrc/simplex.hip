// Downhill simplex along caustic-centred lines on gfx950.
//
// Sec. 4.2 of McDougall & Albrow 2015 treats each (r, phi) trajectory as one GPU block
// that runs a downhill simplex (Nelder & Mead) for the chi-square minimum, the block's
// threads computing the per-point contributions at every step.  Here one 256-lane
// workgroup takes one (line, map) pair: it keeps the three vertices of a simplex over
// x = (t0', ln tE) (t0' the time of closest approach to the caustic centre) in
// registers, identical on every lane, and evaluates each vertex's chi-square with the
// lanes over the light-curve points (four per lane and pass, their loads in flight
// together; light curves of up to 3072 points are first copied to LDS): binary32 samples as in the search, FP64 sums of the centred one-pass fit
// (w b, w b^2, b w (F - Fbar) with b = A - 1) combined in a fixed order (wavefront
// reduce-scatter, then the four wavefronts in order), and a direct second pass of
// w r^2 when the fit is degenerate or flagged as cancellation-prone.  The simplex steps
// follow the standard coefficients (reflection 1, expansion 2, contraction 1/2, shrink
// 1/2) with the acceptance rules of Lagarias et al. (1998); the vertices are kept
// ordered by a stable sort (a new vertex ranks after old ones of equal value; NaN
// counts as +inf).  The steps form a state machine around a single chi-square call,
// and all control flow is uniform across the workgroup, since every lane holds the
// same sums.

#include "simplex.h"

namespace morse {

namespace {

constexpr int kItemThreads = 256;  // one workgroup (four wavefronts) per (line, map)
constexpr int kItemWaves = kItemThreads / kWave;
constexpr int kUnroll = 4;  // points per lane and iteration of a chi-square pass
constexpr int kStagePoints = 3072;  // light curves up to this length go to LDS (60 KiB)

struct Vertex {
  double x0, x1, f;
};

__device__ __forceinline__ void order3(Vertex (&v)[3]) {
  for (int i = 1; i < 3; ++i)
    for (int j = i; j > 0 && v[j].f < v[j - 1].f; --j) {
      const Vertex t = v[j];
      v[j] = v[j - 1];
      v[j - 1] = t;
    }
}

// Sum of N FP64 values over the workgroup: wavefront reduce-scatter, then the wave
// partials in wave order; every thread returns the same values.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double (*s_red)[4]) {
  wave_sums<N>(v);
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0)
    for (int q = 0; q < N; ++q) s_red[wave][q] = v[q];
  __syncthreads();
  for (int q = 0; q < N; ++q) {
    double t = s_red[0][q];
    for (int k = 1; k < kItemWaves; ++k) t += s_red[k][q];
    v[q] = t;
  }
  __syncthreads();
}

// With kStaged the light curve's t, w and w (F - Fbar) are copied to LDS once per
// workgroup (n_points <= kStagePoints) and every evaluation reads them from there.
template <bool kStaged>
__global__ __launch_bounds__(kItemThreads) void k_line_simplex(SimplexArgs a) {
  __shared__ double s_red[kItemWaves][4];
  __shared__ float s_t[kStaged ? kStagePoints : 1];
  __shared__ double s_w[kStaged ? kStagePoints : 1], s_f[kStaged ? kStagePoints : 1];
  const int tid = threadIdx.x;
  const int64_t items = a.n_lines * a.n_maps;
  const int32_t e = a.event;
  const int64_t p0 = uniform(a.lc.off[e]);
  const int32_t np = (int32_t)(uniform(a.lc.off[e + 1]) - p0);
  const float* t = a.lc.t + p0;
  const double* w = a.lc.w + p0;
  const double* wFc = a.lc.wFc + p0;
  const double* F = a.lc.F + p0;
  if (kStaged) {
    for (int32_t i = tid; i < np; i += kItemThreads) {
      s_t[i] = t[i];
      s_w[i] = w[i];
      s_f[i] = wFc[i];
    }
    __syncthreads();
  }
  const double t_ref = uniform(a.lc.t_ref[e]);
  const double Sw = uniform(a.lc.sums[3 * e]), Fbar = uniform(a.lc.sums[3 * e + 1]),
               V = uniform(a.lc.sums[3 * e + 2]);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const int64_t l = a.order ? (int64_t)uniform(a.order[item / a.n_maps]) : item / a.n_maps;
    const int64_t out = l * a.n_maps + item % a.n_maps;
    const MapC m = uniform(a.maps[item % a.n_maps]);
    const double u0 = uniform(a.lines[3 * l]), al = uniform(a.lines[3 * l + 1]),
                 shift = uniform(a.lines[3 * l + 2]);
    double sn, cn;
    sincos(al, &sn, &cn);
    const float ca = (float)cn, sa = (float)sn, bx = (float)(-u0 * sn), by = (float)(u0 * cn);
    auto chi2_at = [&](double x0, double x1) -> double {
      const double tE = exp(x1);
      const double t0 = x0 - shift * tE;
      const float iE = (float)(1.0 / tE);
      const float t0p = (float)(t0 - t_ref);
      double v[3] = {0.0, 0.0, 0.0};
      // four points per lane and iteration, their cells and weights all in flight before
      // the first is added (past the end: clamped loads, never added)
      for (int32_t i0 = tid; i0 < np; i0 += kUnroll * kItemThreads) {
        Loc lc[kUnroll];
        Quad q[kUnroll];
        double wv[kUnroll], fv[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const int32_t j = i0 + k * kItemThreads;
          const uint32_t jj = (uint32_t)(j < np ? j : np - 1);
          lc[k] = locate(m, kStaged ? s_t[jj] : ldg(t, jj), t0p, iE, ca, sa, bx, by);
          q[k] = ldq(m, lc[k].q);
          wv[k] = kStaged ? s_w[jj] : ldg(w, jj);
          fv[k] = kStaged ? s_f[jj] : ldg(wFc, jj);
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          if (i0 + k * kItemThreads >= np) break;
          const float e0 = q[k].v10 - q[k].v00, e1 = q[k].v11 - q[k].v01;
          const float ax0 = q[k].v00 + lc[k].fx * e0, ax1 = q[k].v01 + lc[k].fx * e1;
          const float A = lc[k].on ? ax0 + lc[k].fy * (ax1 - ax0) : point_lens_A(lc[k].zx, lc[k].zy);
          const double b = (double)A - 1.0;
          const double wb = wv[k] * b;
          v[0] += wb;
          v[1] = fma(wb, b, v[1]);
          v[2] = fma(b, fv[k], v[2]);
        }
      }
      block_sums<3>(v, s_red);
      const Fit fit = centred_fit(Sw, Fbar, V, v[0], v[1], v[2], fit_terms(np, kItemThreads));
      double c2 = fit.chi2;
      if (fit.degenerate || fit.recheck) {
        double r2[1] = {0.0}, r2c = 0.0;
        for (int32_t i = tid; i < np; i += kItemThreads) {
          const double A = (double)sample_A(m, t[i], t0p, iE, ca, sa, bx, by);
          const double r = F[i] - fit.Fs * A - fit.Fb;
          neumaier_add(r2[0], r2c, (w[i] * r) * r);
        }
        r2[0] += r2c;
        block_sums<1>(r2, s_red);
        c2 = r2[0];
      }
      return c2 != c2 ? __builtin_inf() : c2;
    };
    // The simplex as a state machine around one chi-square call site: each pass
    // evaluates the pending point (px0, px1), then decides the next one.
    enum { kInit0, kInit1, kInit2, kReflect, kExpand, kContractOut, kContractIn, kShrink1, kShrink2 };
    const double s0 = uniform(a.start[2 * l]), s1 = log(uniform(a.start[2 * l + 1]));
    Vertex v[3];
    double px0 = s0, px1 = s1, b0 = 0.0, b1 = 0.0, r0 = 0.0, r1 = 0.0, fr = 0.0;
    int state = kInit0;
    int32_t it = 0, evals = 0;
    for (;;) {
      const double f = chi2_at(px0, px1);
      ++evals;
      bool next = false;  // an iteration is complete: order, test, start the next
      bool shrink = false;
      switch (state) {
        case kInit0:
          v[0] = {px0, px1, f};
          px0 = s0 + a.d_t0;
          state = kInit1;
          break;
        case kInit1:
          v[1] = {px0, px1, f};
          px0 = s0;
          px1 = s1 + a.d_ln_tE;
          state = kInit2;
          break;
        case kInit2:
          v[2] = {px0, px1, f};
          next = true;
          break;
        case kReflect:
          fr = f;
          if (fr < v[0].f) {
            px0 = b0 + 2.0 * (b0 - v[2].x0);
            px1 = b1 + 2.0 * (b1 - v[2].x1);
            state = kExpand;
          } else if (fr < v[1].f) {
            v[2] = {r0, r1, fr};
            next = true;
          } else if (fr < v[2].f) {
            px0 = b0 + 0.5 * (r0 - b0);
            px1 = b1 + 0.5 * (r1 - b1);
            state = kContractOut;
          } else {
            px0 = b0 + 0.5 * (v[2].x0 - b0);
            px1 = b1 + 0.5 * (v[2].x1 - b1);
            state = kContractIn;
          }
          break;
        case kExpand:
          v[2] = f < fr ? Vertex{px0, px1, f} : Vertex{r0, r1, fr};
          next = true;
          break;
        case kContractOut:
          if (f <= fr) {
            v[2] = {px0, px1, f};
            next = true;
          } else {
            shrink = true;
          }
          break;
        case kContractIn:
          if (f < v[2].f) {
            v[2] = {px0, px1, f};
            next = true;
          } else {
            shrink = true;
          }
          break;
        case kShrink1:
          v[1] = {px0, px1, f};
          px0 = v[0].x0 + 0.5 * (v[2].x0 - v[0].x0);
          px1 = v[0].x1 + 0.5 * (v[2].x1 - v[0].x1);
          state = kShrink2;
          break;
        default:  // kShrink2
          v[2] = {px0, px1, f};
          next = true;
          break;
      }
      if (shrink) {  // towards the best vertex: vertex 1 now, vertex 2 next
        px0 = v[0].x0 + 0.5 * (v[1].x0 - v[0].x0);
        px1 = v[0].x1 + 0.5 * (v[1].x1 - v[0].x1);
        state = kShrink1;
      }
      if (!next) continue;
      order3(v);
      if (it >= a.max_iter || v[2].f - v[0].f <= a.ftol * fabs(v[0].f)) break;
      ++it;
      b0 = (v[0].x0 + v[1].x0) * 0.5;
      b1 = (v[0].x1 + v[1].x1) * 0.5;
      r0 = b0 + (b0 - v[2].x0);
      r1 = b1 + (b1 - v[2].x1);
      px0 = r0;
      px1 = r1;
      state = kReflect;
    }
    if (tid == 0) {
      a.chi2[out] = v[0].f;
      a.t0[out] = v[0].x0;
      a.tE[out] = exp(v[0].x1);
      a.iters[out] = it;
      if (a.evals) a.evals[out] = evals;
    }
  }
}

// One wavefront per line: the largest sample along it on the first map (as the line
// filter samples), as a descending log2 bucket (NaN and non-positive maxima last).
__global__ __launch_bounds__(256) void k_simplex_prio(SimplexArgs a, double cxw, double cyw,
                                                      double half_diag, int32_t ns, float h,
                                                      uint32_t* key) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const MapC m = uniform(a.maps[0]);
  for (int64_t l = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; l < a.n_lines;
       l += waves) {
    const double u0 = a.lines[3 * l], al = a.lines[3 * l + 1];
    double sn, cn;
    sincos(al, &sn, &cn);
    const float ca = (float)cn, sa = (float)sn, bx = (float)(-u0 * sn), by = (float)(u0 * cn);
    const float lo = (float)((cxw * cn + cyw * sn) - half_diag);
    float best = 0.0f;
    for (int k = lane; k < ns; k += kWave) {
      const float A = sample_A(m, lo + (float)k * h, 0.0f, 1.0f, ca, sa, bx, by);
      best = A > best ? A : best;  // NaN samples never win
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) best = fmaxf(best, __shfl_xor(best, off));
    if (lane == 0) {
      int b = 0;  // bucket of log2(best) over [2^-8, 2^13.3), 48 per octave
      if (best > 0.0f) b = min(max((int)((log2f(best) + 8.0f) * 48.0f), 0), kSimplexPrioBins - 1);
      key[l] = (uint32_t)(kSimplexPrioBins - 1 - b);
    }
  }
}

}  // namespace

hipError_t launch_simplex_order(const SimplexArgs& a, double cxw, double cyw, double half_diag,
                                int32_t ns, float h, uint32_t* key, uint32_t* hist, int32_t* order,
                                hipStream_t st) {
  if (a.n_lines <= 0) return hipSuccess;
  if (a.n_lines > INT32_MAX || ns < 1 || a.n_maps < 1) return hipErrorInvalidValue;
  int64_t blocks = (a.n_lines + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_simplex_prio, dim3((unsigned)blocks), dim3(256), 0, st, a, cxw, cyw, half_diag,
                     ns, h, key);
  return launch_bucket_order(key, a.n_lines, kSimplexPrioBins, hist, order, st);
}

hipError_t launch_line_simplex(const SimplexArgs& a, hipStream_t st) {
  const int64_t items = a.n_lines * a.n_maps;
  if (items <= 0) return hipSuccess;
  int64_t blocks = items;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (a.n_points <= kStagePoints)
    hipLaunchKernelGGL(k_line_simplex<true>, dim3((unsigned)blocks), dim3(kItemThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_line_simplex<false>, dim3((unsigned)blocks), dim3(kItemThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace morse
