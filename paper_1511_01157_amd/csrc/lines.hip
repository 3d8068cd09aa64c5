// Caustic-centred trajectory lines on gfx950: the minimum-magnification filter and the
// expansion of the kept lines into trajectory lists.
//
// Sec. 4.2 of McDougall & Albrow 2015 searches straight trajectories at radial distances
// from the caustic centres; sec. 4.3 first discards every trajectory whose magnification
// along its path, read from the point-source map, stays below the minimum that the
// light curve implies.  A line here is (u0, alpha, shift): the path tau (cos a, sin a) +
// u0 (-sin a, cos a), whose closest approach to its caustic centre is at tau = shift.
//
// Filter layout.  One wavefront per line, lanes over the samples: the line is sampled
// across the map window at spacing h <= 1 pixel, each sample exactly as the search
// samples a point (the same binary32 geometry and bilinear blend of the packed cells,
// the single-lens value off the map), and the largest value (NaN if any sample is NaN)
// decides.  The kept lines are then listed in ascending order by a three-step
// stream compaction (counts per block, one scan, scatter), so the result does not
// depend on the schedule.

#include "lines.h"

namespace morse {

namespace {

constexpr int kFilterThreads = 256;
constexpr int kCompactThreads = 256;
constexpr int kCompactPer = 4;  // flags per thread
constexpr int kCompactBlock = kCompactThreads * kCompactPer;

constexpr float kInf = __builtin_inff();

// lane j's value, the same in every lane (j uniform)
__device__ __forceinline__ float lane_at(float v, int32_t j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// max that propagates NaN (as a maximum over an array does)
__device__ __forceinline__ float nanmax(float a, float b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

__global__ __launch_bounds__(kFilterThreads) void k_line_filter(LineFilterArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (kFilterThreads / kWave);
  for (int64_t l = blockIdx.x * (int64_t)(kFilterThreads / kWave) + threadIdx.x / kWave; l < a.n;
       l += waves) {
    const double u0 = a.lines[3 * l], al = a.lines[3 * l + 1];
    double sn, cn;
    sincos(al, &sn, &cn);
    const float ca = (float)cn, sa = (float)sn;
    const float bx = (float)(-u0 * sn), by = (float)(u0 * cn);
    const double tau_c = a.cxw * cn + a.cyw * sn;
    const float lo = (float)(tau_c - a.half_diag);
    float best = -__builtin_inff();
    for (int k = lane; k < a.ns; k += kWave) {
      const float tau = lo + (float)k * a.h;
      best = nanmax(best, sample_A(a.m, tau, 0.0f, 1.0f, ca, sa, bx, by));
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) best = nanmax(best, __shfl_xor(best, off));
    if (lane == 0) {
      a.best[l] = best;
      a.keep[l] = best >= a.amin ? 1 : 0;
    }
  }
}

// Inclusive prefix over the wavefront's lanes (Hillis-Steele): lane j gets the
// combination of lanes 0..j.  kMin keeps the left value unless the right is smaller,
// otherwise unless the right is larger, so among equal values the leftmost survives;
// the keys hold no NaN, which makes either combination associative.
template <bool kMin>
__device__ __forceinline__ float lane_prefix(float x, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const float l = __shfl_up(x, d);
    if (lane >= d) x = (kMin ? (x < l) : (x > l)) ? x : l;
  }
  return x;
}

// Peak library.  One wavefront per line (four per workgroup): each chunk of 64 samples is
// computed lane-parallel exactly as in the filter.  A peak is a rise above fl32(trough *
// up) followed by a fall below fl32(top * down); the first sample starts the first
// trough; equal maxima keep the first.  The rule is a left-to-right scan, but between
// two of its events (a rise, a fall) the state changes only by a running minimum (the
// trough) or a running maximum (the top and its index), so each chunk is taken one
// event at a time: a prefix minimum or maximum over the lanes gives every sample the
// trough or top the scan would hold before it, the first lane whose sample rises or
// falls against that value (found by ballot) is the next event, and the scan resumes
// after it.  A chunk costs one prefix per event plus one, not one step per sample.  NaN
// samples neither lower the trough, raise the top nor trigger an event, as in the
// scan; a NaN first sample leaves the trough NaN and the line without peaks.
__global__ __launch_bounds__(kFilterThreads) void k_line_peaks(LinePeakArgs a) {
  const LineFilterArgs& f = a.f;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (kFilterThreads / kWave);
  const float nan = __builtin_nanf("");
  for (int64_t l = blockIdx.x * (int64_t)(kFilterThreads / kWave) + threadIdx.x / kWave; l < f.n;
       l += waves) {
    const double u0 = f.lines[3 * l], al = f.lines[3 * l + 1];
    double sn, cn;
    sincos(al, &sn, &cn);
    const float ca = (float)cn, sa = (float)sn;
    const float bx = (float)(-u0 * sn), by = (float)(u0 * cn);
    const double tau_c = f.cxw * cn + f.cyw * sn;
    const float lo = (float)(tau_c - f.half_diag);
    float best = -__builtin_inff();
    float trough = 0.0f, top = 0.0f;
    int32_t top_i = 0, count = 0;
    bool rising = false;
    for (int32_t c0 = 0; c0 < f.ns; c0 += kWave) {
      const int32_t k = c0 + lane;
      float A = nan;
      if (k < f.ns) {
        A = sample_A(f.m, lo + (float)k * f.h, 0.0f, 1.0f, ca, sa, bx, by);
        best = nanmax(best, A);
      }
      const int32_t nk = min(kWave, f.ns - c0);
      int32_t s = 0;  // first sample of the chunk not yet scanned
      if (c0 == 0) {
        trough = lane_at(A, 0);
        s = 1;
      }
      const bool real = lane < nk && A == A;
      while (s < nk) {
        const bool act = lane >= s && lane < nk;
        if (!rising) {
          if (trough != trough) break;  // no sample compares with a NaN trough
          const float p = lane_prefix<true>(act && real ? A : kInf, lane);
          float T = __shfl_up(p, 1);
          if (lane == 0) T = kInf;
          T = T < trough ? T : trough;  // the trough before this lane's sample
          const uint64_t ev = __builtin_amdgcn_ballot_w64(act && !(A < T) && A > T * a.up);
          if (ev == 0) {
            const float m = lane_at(p, nk - 1);
            if (m < trough) trough = m;
            break;
          }
          const int32_t j = __builtin_ctzll(ev);
          top = lane_at(A, j);
          top_i = c0 + j;
          rising = true;
          s = j + 1;
        } else {
          const float p = lane_prefix<false>(act && real ? A : -kInf, lane);
          float T = __shfl_up(p, 1);
          if (lane == 0) T = -kInf;
          T = T > top ? T : top;  // the top before this lane's sample
          const uint64_t ev = __builtin_amdgcn_ballot_w64(act && !(A > T) && A < T * a.down);
          const int32_t end = ev ? __builtin_ctzll(ev) : nk;  // samples s .. end-1 precede it
          if (end > s) {
            const float m = lane_at(p, end - 1);
            if (m > top) {  // the first sample equal to the new maximum
              const int32_t j = __builtin_ctzll(
                  __builtin_amdgcn_ballot_w64(lane >= s && lane < end && A == m));
              top = lane_at(A, j);
              top_i = c0 + j;
            }
          }
          if (ev == 0) break;
          if (lane == 0 && count < a.kmax) {
            a.ptau[l * a.kmax + count] = lo + (float)top_i * f.h;
            a.pA[l * a.kmax + count] = top;
          }
          ++count;
          rising = false;
          trough = lane_at(A, end);
          s = end + 1;
        }
      }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) best = nanmax(best, __shfl_xor(best, off));
    for (int32_t j = count + lane; j < a.kmax; j += kWave) {
      a.ptau[l * a.kmax + j] = nan;
      a.pA[l * a.kmax + j] = nan;
    }
    if (lane == 0) {
      f.best[l] = best;
      a.npeaks[l] = count;
      f.keep[l] = (best >= f.amin && count >= a.min_peaks) ? 1 : 0;
    }
  }
}

// Eqs. 7-8 per line, in FP64: one observed time -> the highest peak (ties: the earlier)
// with the given tE; two -> the two highest, in tau order.  t0' = t0 + shift tE.
__global__ __launch_bounds__(256) void k_peak_starts(PeakStartArgs a) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = a.kept ? a.kept[k] : k;
    const int32_t np = min(a.npeaks[l], a.kmax);
    double s0 = __builtin_nan(""), s1 = __builtin_nan("");
    if (np >= a.n_tp) {
      const float* A = a.pA + l * a.kmax;
      const float* T = a.ptau + l * a.kmax;
      int32_t j1 = 0;  // highest
      for (int32_t j = 1; j < np; ++j)
        if (A[j] > A[j1]) j1 = j;
      const double shift = a.lines[3 * l + 2];
      double tE, t0;
      if (a.n_tp == 1) {
        tE = a.tE;
        t0 = a.tp1 - (double)T[j1] * tE;
      } else {
        int32_t j2 = -1;  // second highest
        for (int32_t j = 0; j < np; ++j)
          if (j != j1 && (j2 < 0 || A[j] > A[j2])) j2 = j;
        const int32_t lo = min(j1, j2), hi = max(j1, j2);
        const double m1 = (double)T[lo], m2 = (double)T[hi];
        tE = (a.tp2 - a.tp1) / (m2 - m1);
        t0 = a.tp1 - m1 * tE;
      }
      s0 = t0 + shift * tE;
      s1 = tE;
    }
    a.start[2 * k] = s0;
    a.start[2 * k + 1] = s1;
  }
}

// Block b counts the set flags of keep[b B, (b + 1) B).
__global__ __launch_bounds__(kCompactThreads) void k_compact_count(const uint8_t* keep, int64_t n,
                                                                   int64_t* counts) {
  __shared__ int s[kCompactThreads];
  const int64_t base = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x * kCompactPer;
  int c = 0;
  for (int j = 0; j < kCompactPer; ++j)
    if (base + j < n) c += keep[base + j] ? 1 : 0;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int w = kCompactThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// Exclusive scan of the nb block counts in place (one workgroup, chunk by chunk); the
// total goes to *total.
__global__ __launch_bounds__(kCompactThreads) void k_compact_scan(int64_t* counts, int64_t nb,
                                                                  int64_t* total) {
  __shared__ int64_t s[kCompactThreads];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kCompactThreads) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? counts[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < kCompactThreads; w <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) counts[i] = carry + s[threadIdx.x] - v;
    carry += s[kCompactThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// Block b writes the indices of its set flags from position offsets[b] on.
__global__ __launch_bounds__(kCompactThreads) void k_compact_scatter(const uint8_t* keep, int64_t n,
                                                                     const int64_t* offsets,
                                                                     int64_t* kept) {
  __shared__ int s[kCompactThreads];
  const int64_t base = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x * kCompactPer;
  int c = 0;
  for (int j = 0; j < kCompactPer; ++j)
    if (base + j < n) c += keep[base + j] ? 1 : 0;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int w = 1; w < kCompactThreads; w <<= 1) {
    const int add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t pos = offsets[blockIdx.x] + s[threadIdx.x] - c;
  for (int j = 0; j < kCompactPer; ++j)
    if (base + j < n && keep[base + j]) kept[pos++] = base + j;
}

__global__ __launch_bounds__(256) void k_lines_traj(const double* lines, const int64_t* kept,
                                                    int64_t n_kept, const double* t0, int32_t n_t0,
                                                    const double* tE, int32_t n_tE,
                                                    double* params) {
  const int64_t per = (int64_t)n_t0 * n_tE;
  const int64_t total = n_kept * per;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = j / per;
    const int32_t a = (int32_t)((j / n_tE) % n_t0), b = (int32_t)(j % n_tE);
    const int64_t l = kept ? kept[k] : k;
    const double u0 = lines[3 * l], al = lines[3 * l + 1], shift = lines[3 * l + 2];
    params[4 * j] = t0[a] - shift * tE[b];
    params[4 * j + 1] = u0;
    params[4 * j + 2] = tE[b];
    params[4 * j + 3] = al;
  }
}

}  // namespace

hipError_t launch_line_filter(const LineFilterArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (!a.lines || !a.best || !a.keep || a.ns < 2 || !a.m.quad) return hipErrorInvalidValue;
  const int64_t per_block = kFilterThreads / kWave;
  int64_t blocks = (a.n + per_block - 1) / per_block;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(k_line_filter, dim3((unsigned)blocks), dim3(kFilterThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_line_peaks(const LinePeakArgs& a, hipStream_t st) {
  if (a.f.n <= 0) return hipSuccess;
  if (!a.f.lines || !a.f.best || !a.f.keep || !a.npeaks || !a.ptau || !a.pA || a.f.ns < 2 ||
      !a.f.m.quad || a.kmax < 1)
    return hipErrorInvalidValue;
  const int64_t per_block = kFilterThreads / kWave;
  int64_t blocks = (a.f.n + per_block - 1) / per_block;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(k_line_peaks, dim3((unsigned)blocks), dim3(kFilterThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_peak_starts(const PeakStartArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  int64_t blocks = (a.n + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(k_peak_starts, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t compact_scratch_elems(int64_t n) { return (size_t)((n + kCompactBlock - 1) / kCompactBlock) + 1; }

hipError_t launch_compact(const uint8_t* keep, int64_t n, int64_t* scratch, int64_t* kept,
                          int64_t* d_count, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  const int64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
  if (nb > (int64_t)1 << 30) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_compact_count, dim3((unsigned)nb), dim3(kCompactThreads), 0, st, keep, n,
                     scratch);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kCompactThreads), 0, st, scratch, nb, d_count);
  if (kept)
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)nb), dim3(kCompactThreads), 0, st, keep,
                       n, scratch, kept);
  return hipGetLastError();
}

hipError_t launch_lines_to_traj(const double* lines, const int64_t* kept, int64_t n_kept,
                                const double* t0, int32_t n_t0, const double* tE, int32_t n_tE,
                                double* params, hipStream_t st) {
  const int64_t total = n_kept * (int64_t)n_t0 * n_tE;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(k_lines_traj, dim3((unsigned)blocks), dim3(256), 0, st, lines, kept, n_kept,
                     t0, n_t0, tE, n_tE, params);
  return hipGetLastError();
}

}  // namespace morse
