// Internal declarations of the gfx950 library: device-side data layouts, the
// per-sample arithmetic shared by the search and gradient kernels, and the host
// launchers each kernel file exports to the C ABI sources (api_*.hip).  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/morse.h"

namespace morse {

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------------------
// Ray shooting constants, each rounded once from FP64 to binary32 on the host.
struct RayParams {
  float m1, m2, x1, x2;  // lens masses and positions
  float cx, cy, hx, hy;  // lattice centre and spacing
  float sx, sy, kx, ky;  // window centre and pixels per Einstein radius
  int32_t nx, ny, mx, my;
  int32_t row0, row1;    // lattice rows [row0, row1)
};

// Per-trajectory constants: binary32 geometry rounded once from FP64, t0 kept FP64
// so each event subtracts its own reference time before rounding.
struct TrajC {
  double t0;
  float iE, ca, sa, bx, by, pad;
};
static_assert(sizeof(TrajC) == 32, "TrajC layout");

// A map as the sampling kernels see it.  The row-major pixel values `map` are packed
// once per call into `quad`: cell (i, j), 0 <= i < mx - 1, 0 <= j < my - 1, holds the
// four pixel-centre values (A[j][i], A[j][i+1], A[j+1][i], A[j+1][i+1]) as one 16-byte
// Quad, and the cells are grouped in tiles of 4 (x) by 2 (y) cells, one 128-byte
// cache line each, tiles in row-major order, cells inside a tile column-major:
//   q(i, j) = ((j / 2) (4 tiles_x) + i) 2 + j % 2
// (= 8 tile + 2 (i % 4) + j % 2, tile = (j / 2) tiles_x + i / 4), so the byte offset
// is one 24-bit multiply-add and two shifts.  A bilinear sample is then one aligned
// load, and the samples of a wavefront along a trajectory touch about 2.5x fewer
// cache lines than two row-major row loads.
// One packed cell: the four pixel-centre values around it.
struct alignas(16) Quad {
  float v00, v10, v01, v11;
};

struct MapC {
  const float* map;
  const Quad* quad;
  uint32_t tiles_x, tiles_y;
  int32_t mx, my;
  float sx, sy, kx, ky, ox, oy;  // grid coordinate g = (zeta - s) k + o
  float lx, ly;                  // on-map bound: g < M - 1
};
// Load of the cell at byte offset qb: one buffer_load_dwordx4 through a raw buffer
// resource over the map's packed cells.  The resource is uniform (scalar registers) and
// the offset one 32-bit register, so a load needs no 64-bit address arithmetic, and an
// offset outside the packed map reads zeros instead of faulting (the hardware range
// check).  Word 3 of the resource: data format 32 bits (bits 15-18 = 4), nothing else.
constexpr int kRawBufferWord3 = 0x00020000;
__device__ __forceinline__ Quad ldq(const MapC& m, uint32_t qb) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  // tiles_x tiles_y 128 < 2^32: the host rejects larger packed maps
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      (void*)m.quad, (short)0, (int)(m.tiles_x * m.tiles_y * 128u), kRawBufferWord3);
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)qb, 0, 0);
  return Quad{__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
              __uint_as_float(v.w)};
}

// Packed size of a map with mx x my pixels (bytes).
inline size_t quad_bytes(int32_t mx, int32_t my) {
  return (size_t)((mx - 1 + 3) / 4) * (size_t)((my - 1 + 1) / 2) * 128;
}

// Light curves after preparation: per point binary32 time offset, w and the
// centred weighted flux w (F - Fbar); per event S_w, the weighted mean Fbar and
// V = sum w (F - Fbar)^2.
struct LcView {
  const float* t;
  const double* w;
  const double* wFc;
  const double* F;
  const int64_t* off;   // device CSR offsets [n_events + 1]
  const double* sums;   // [n_events][3]: S_w, Fbar, V
  const double* t_ref;  // [n_events]
};

// ---------------------------------------------------------------------------
// Sampling along a trajectory (binary32, no fused multiply-add: the library is
// compiled with -ffp-contract=off, so every operation below rounds on its own).
//   tau = (t - t0')*iE; zeta = tau (ca, sa) + (bx, by); g = (zeta - s) k + o;
//   bilinear between pixel-centre values inside [0, M-1), else the single-lens
//   magnification (uu + 2)/sqrt(uu (uu + 4)) about the barycentre.
struct Sample {
  float A;
  float tau, zx, zy;
  float fx, fy, e0, e1, ax0, ax1;
  bool on;
};

// Load base[i] through a uniform base pointer and a 32-bit element offset, so the
// backend can address with a scalar base plus one 32-bit VGPR offset.  The pointer is
// taken as global memory explicitly (a pointer rebuilt from scalar registers has lost
// its address space, and a generic pointer would compile to a slower flat load).
template <class T>
__device__ __forceinline__ T ldg(const T* __restrict__ base, uint32_t i) {
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) T gT;
  return *(gT*)((gchar*)base + (size_t)(i * (uint32_t)sizeof(T)));
}

// Byte offset of packed cell (i, j); (j / 2) (4 tiles_x) + i < 2^27 since the packed
// map is below 4 GiB, and both factors fit 24 bits.
__device__ __forceinline__ uint32_t cell_offset(const MapC& m, uint32_t i, uint32_t j) {
  return ((__umul24(j >> 1, m.tiles_x << 2) + i) << 5) | ((j & 1u) << 4);
}

__device__ __forceinline__ void map_cell(const MapC& m, float fi, float fj, float& v00, float& v10,
                                         float& v01, float& v11) {
  const Quad v = ldq(m, cell_offset(m, (uint32_t)(int)fi, (uint32_t)(int)fj));
  v00 = v.v00;
  v10 = v.v10;
  v01 = v.v01;
  v11 = v.v11;
}

// Sampling in steps, so that the loads of several points can all be issued before
// any of them is used: locate (trajectory position, on-map test, cell), one 16-byte
// fetch of the cell (an off-map lane reads cell 0, and ignores it), then the blend.
// The arithmetic is that of sample_A / sample_full.
struct Loc {
  float tau, zx, zy, fx, fy;
  uint32_t q;  // byte offset of the packed cell (0 off the map)
  bool on;
};

__device__ __forceinline__ Loc locate(const MapC& m, float tt, float t0p, float iE, float ca,
                                      float sa, float bx, float by) {
  Loc l;
  l.tau = (tt - t0p) * iE;
  l.zx = l.tau * ca + bx;
  l.zy = l.tau * sa + by;
  const float gx = ((l.zx - m.sx) * m.kx) + m.ox;
  const float gy = ((l.zy - m.sy) * m.ky) + m.oy;
  // On the map: 0 <= g < M - 1, tested on the bit patterns as unsigned integers (for
  // a positive bound L, bits(g) < bits(L) iff +0 <= g < L; negative values and NaN
  // have larger patterns).  Only g = -0 would differ, and g is a sum with the nonzero
  // constant o = M/2 - 1/2, which an IEEE sum never rounds to -0.
  l.on = ((unsigned)(__float_as_uint(gx) < __float_as_uint(m.lx)) &
          (unsigned)(__float_as_uint(gy) < __float_as_uint(m.ly))) != 0u;
  // on the map g >= 0, so truncation is the floor and fract(g) = g - floor(g) exactly
  l.fx = __builtin_amdgcn_fractf(gx);
  l.fy = __builtin_amdgcn_fractf(gy);
  l.q = l.on ? cell_offset(m, (uint32_t)gx, (uint32_t)gy) : 0u;
  return l;
}

// Single-lens magnification about the barycentre, (uu + 2)/sqrt(uu (uu + 4)), with a
// correctly rounded binary32 square root and quotient.  A correctly rounded result is
// unique, so any exact method gives the same bits.  When d = uu (uu + 4) lies in
// [2^-60, 2^60] on every active lane the short form runs: the hardware square root
// (within one ulp) corrected by the signs of the FMA residuals against its two
// neighbours, then the reciprocal refined once and the quotient corrected twice by FMA.
// These are the steps of the general IEEE sequences with their range scalings and
// special-case fix-ups left out, which in this range change nothing.  Elsewhere the
// general sequences run.
__device__ __forceinline__ float point_lens_A(float zx, float zy) {
  const float uu = zx * zx + zy * zy;
  const float p = uu + 2.0f, d = uu * (uu + 4.0f);
  if (__builtin_amdgcn_ballot_w64(!(d >= 0x1p-60f && d <= 0x1p60f)) == 0) {
    float s = __builtin_amdgcn_sqrtf(d);
    const float sdn = __uint_as_float(__float_as_uint(s) - 1u);
    const float sup = __uint_as_float(__float_as_uint(s) + 1u);
    const float rdn = fmaf(-sdn, s, d), rup = fmaf(-sup, s, d);
    s = rdn <= 0.0f ? sdn : s;
    s = rup > 0.0f ? sup : s;
    float r = __builtin_amdgcn_rcpf(s);
    r = fmaf(fmaf(-s, r, 1.0f), r, r);
    float q = p * r;
    q = fmaf(fmaf(-s, q, p), r, q);
    return fmaf(fmaf(-s, q, p), r, q);
  }
  return p / sqrtf(d);
}

__device__ __forceinline__ float sample_A(const MapC& m, float tt, float t0p, float iE, float ca,
                                          float sa, float bx, float by) {
  const float tau = (tt - t0p) * iE;
  const float zx = tau * ca + bx;
  const float zy = tau * sa + by;
  const float gx = ((zx - m.sx) * m.kx) + m.ox;
  const float gy = ((zy - m.sy) * m.ky) + m.oy;
  if (gx >= 0.0f && gx < m.lx && gy >= 0.0f && gy < m.ly) {
    const float fi = floorf(gx);
    const float fj = floorf(gy);
    const float fx = gx - fi;
    const float fy = gy - fj;
    float v00, v10, v01, v11;
    map_cell(m, fi, fj, v00, v10, v01, v11);
    const float e0 = v10 - v00;
    const float e1 = v11 - v01;
    const float ax0 = v00 + fx * e0;
    const float ax1 = v01 + fx * e1;
    return ax0 + fy * (ax1 - ax0);
  }
  const float uu = zx * zx + zy * zy;
  return (uu + 2.0f) / sqrtf(uu * (uu + 4.0f));
}

__device__ __forceinline__ Sample sample_full(const MapC& m, float tt, float t0p, float iE,
                                              float ca, float sa, float bx, float by) {
  Sample s;
  s.tau = (tt - t0p) * iE;
  s.zx = s.tau * ca + bx;
  s.zy = s.tau * sa + by;
  const float gx = ((s.zx - m.sx) * m.kx) + m.ox;
  const float gy = ((s.zy - m.sy) * m.ky) + m.oy;
  s.on = (gx >= 0.0f && gx < m.lx && gy >= 0.0f && gy < m.ly);
  if (s.on) {
    const float fi = floorf(gx);
    const float fj = floorf(gy);
    s.fx = gx - fi;
    s.fy = gy - fj;
    float v00, v10, v01, v11;
    map_cell(m, fi, fj, v00, v10, v01, v11);
    s.e0 = v10 - v00;
    s.e1 = v11 - v01;
    s.ax0 = v00 + s.fx * s.e0;
    s.ax1 = v01 + s.fx * s.e1;
    s.A = s.ax0 + s.fy * (s.ax1 - s.ax0);
  } else {
    const float uu = s.zx * s.zx + s.zy * s.zy;
    s.A = (uu + 2.0f) / sqrtf(uu * (uu + 4.0f));
    s.fx = s.fy = s.e0 = s.e1 = s.ax0 = s.ax1 = 0.0f;
  }
  return s;
}

// A value known to be the same on every lane, moved to scalar registers word by word
// (loads from memory the kernel also writes are vector loads, whose results the
// compiler would otherwise keep in vector registers).
template <class T>
__device__ __forceinline__ T uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "uniform() moves 32-bit words");
  T r;
  const int* src = reinterpret_cast<const int*>(&v);
  int* dst = reinterpret_cast<int*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return r;
}

// Deterministic wavefront sum (butterfly over 64 lanes, same order on every lane).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Wavefront reduce-scatter of N FP64 values per lane.  Each halving step over lane
// bit MASK keeps ceil(N/2) slots: lanes with the bit set keep the upper half (padded
// with a zero), the others the lower half, each adding its partner's copy of the slots
// it keeps; six steps (MASK = 32 .. 1) exchange about N values in all, against 6 N for
// one butterfly per value.  Each value is summed over the same pairing tree as
// wave_sum (IEEE addition commutes), so the totals are bitwise those of wave_sum.  On
// return v[0] holds the total of original value `slot` when `valid`; every value
// appears on exactly one valid lane, rs_lane<N>(q).
template <int N, int MASK = 32>
__device__ __forceinline__ void reduce_scatter(double* v, int lane, int& slot, bool& valid) {
  if constexpr (MASK >= 1) {
    constexpr int H = (N + 1) / 2;
    const bool up = (lane & MASK) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double lo = v[i];
      const double hi = (i + H < N) ? v[i + H] : 0.0;
      const double other = __shfl_xor(up ? lo : hi, MASK, kWave);
      v[i] = (up ? hi : lo) + other;
    }
    reduce_scatter<H, MASK / 2>(v, lane, slot, valid);
    slot += up ? H : 0;
    valid = valid && slot < N;
  }
}

// Lane that holds value q after reduce_scatter<N>.
template <int N>
constexpr int rs_lane(int q) {
  int lane = 0, n = N;
  for (int mask = 32; mask >= 1; mask >>= 1) {
    const int h = (n + 1) / 2;
    if (q >= h) {
      lane |= mask;
      q -= h;
    }
    n = h;
  }
  return lane;
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wavefront totals of N values, on every lane (bitwise wave_sum of each value).
template <int N>
__device__ __forceinline__ void wave_sums(double (&v)[N]) {
  int slot = 0;
  bool valid = true;
  reduce_scatter<N>(v, threadIdx.x & (kWave - 1), slot, valid);
  const double mine = v[0];
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = read_lane(mine, rs_lane<N>(q));
}

// Neumaier's compensated addition: s + c carries the sum, c the rounding errors.
__device__ __forceinline__ void neumaier_add(double& s, double& c, double v) {
  double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// Profiled fit (Eqs. 5-6) in centred form.  With b = A - 1 and per-point
// wFc = w (F - Fbar), one pass gives B1 = sum w b, B2 = sum w b^2, C = sum b wFc.
// Then S_bb = B2 - B1^2/S_w equals det/S_w of the normal equations
// (det = S_AA S_w - S_A^2, S_AA = B2 + 2 B1 + S_w), and
//   F_s = C / S_bb,  F_b = Fbar - F_s (1 + B1/S_w),  chi2 = V - F_s C.
// Degenerate (det <= 1e-12 S_AA S_w, i.e. S_bb <= 1e-12 S_AA): F_s = 0, F_b = Fbar,
// chi2 = V.
//
// The sums are plain (uncompensated) FP64, so the one-pass chi2 comes with a worst-case
// error bound, and `recheck` is set when that bound exceeds 1e-8 chi2; the caller then
// sums w r^2 directly (Neumaier-compensated second pass).  Each of B1, B2, C is a
// recursive sum over one lane's points followed by a fixed reduction tree, so with n
// = the terms per lane + the tree depth + the roundings of one term (fit_terms), its
// error is at most n u sum|terms| (u = 2^-53; Higham, Accuracy and Stability of
// Numerical Algorithms, sec. 4.2), and by Cauchy-Schwarz sum|w b| <= sqrt(S_w B2),
// sum|b wFc| <= sqrt(B2 V).  Through chi2 = V - C^2/S_bb, with F_s^2 S_bb <= V and
// kappa = B2/S_bb >= 1 (V carries its own compensated error, u V):
//   |d chi2| <= u V (n (3 kappa + 2 sqrt(kappa)) + 6 kappa + 5).
// For noisy data chi2 is near the number of points and the bound stays far below the
// threshold; a near-perfect or ill-conditioned fit takes the second pass.
struct Fit {
  double Fs, Fb, chi2;
  bool degenerate, recheck;
};

// Terms per lane plus reduction depth for the bound above: np points over `lanes`
// lanes, a tree of at most 8 levels, at most 2 serial cross-wave additions and 2
// roundings per term.
__device__ __forceinline__ double fit_terms(int32_t np, int lanes) {
  return (double)((np + lanes - 1) / lanes + 12);
}

__device__ __forceinline__ Fit centred_fit(double Sw, double Fbar, double V, double B1, double B2,
                                           double C, double nterms) {
  Fit f;
  const double SAA = (B2 + 2.0 * B1) + Sw;
  const double Sbb = B2 - (B1 * B1) / Sw;
  f.degenerate = !(Sbb > 1e-12 * SAA);
  f.recheck = false;
  if (f.degenerate) {
    f.Fs = 0.0;
    f.Fb = Fbar;
    f.chi2 = V;
    return f;
  }
  f.Fs = C / Sbb;
  f.Fb = Fbar - f.Fs * (1.0 + B1 / Sw);
  f.chi2 = V - f.Fs * C;
  const double kappa = B2 / Sbb;
  const double bound = (nterms * (3.0 * kappa + 2.0 * sqrt(kappa)) + 6.0 * kappa + 5.0) * V;
  f.recheck = !(f.chi2 > 0.0) || (bound > 9.007199254740992e7 * f.chi2);  // 1e-8 / u
  return f;
}

// ---------------------------------------------------------------------------
// Host launchers (one per kernel family); all enqueue on `st` and return the
// first HIP error.
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t st);
// Exclusive prefix sum of nb uint32 counters in place (one workgroup; counting sorts).
hipError_t launch_scan_u32(uint32_t* v, int64_t nb, hipStream_t st);
// order[0 .. n): the items 0 .. n - 1 by ascending key (key < nbins; the order among
// equal keys is unspecified).  hist: nbins counters of workspace.
hipError_t launch_bucket_order(const uint32_t* key, int64_t n, int32_t nbins, uint32_t* hist,
                               int32_t* order, hipStream_t st);
// Packs every map of the device table `maps` (n_maps entries; h_maps the same table on
// the host, for the sizes) into its quad layout.
hipError_t launch_quad_pack(const MapC* maps, const MapC* h_maps, int32_t n_maps, hipStream_t st);
hipError_t launch_rayshoot(const RayParams& p, uint32_t* counts, unsigned long long* stats,
                           hipStream_t st);
// Normalisation + convolution of a counts map with ntaps taps whose offsets reach at
// most rx columns and ry rows from the pixel (rx = ry = 0: the single tap (0, 0);
// otherwise at most 16 each).
hipError_t launch_normalize_convolve(const uint32_t* counts, float* map, int32_t mx, int32_t my,
                                     const float* d_w, const int32_t* d_off, int32_t ntaps,
                                     int32_t rx, int32_t ry, float scale, uint32_t* d_maxc,
                                     hipStream_t st);
hipError_t launch_lc_prep(const float* t, const double* F, const double* w, const int64_t* off,
                          int32_t n_events, double* wF, double* sums, hipStream_t st);
hipError_t launch_traj_prep_list(const double* params, int64_t n, TrajC* out, hipStream_t st);
hipError_t launch_traj_prep_grid(const double* axes, int32_t nu, int32_t na, int32_t nt,
                                 int32_t ne, TrajC* out, hipStream_t st);

struct SearchOut {
  double* chi2;
  double* fs;
  double* fb;
};

// Plain search: one launch for one (event, map); outputs for that segment.
hipError_t launch_search_plain(const TrajC* tc, int64_t n_traj, LcView lc, int32_t event,
                               MapC map, SearchOut out, int waves_per_block, hipStream_t st);

// Batched persistent search over (event, map, trajectory block) items.
struct BatchedArgs {
  const TrajC* tc;          // per event if !shared
  int64_t n_traj;
  int32_t shared;
  int32_t n_events, n_maps;
  const MapC* maps;         // device table [n_maps]
  LcView lc;
  SearchOut out;            // full [e][m][traj] arrays
  uint32_t* counter;        // kQueues work-queue counters, 128 bytes apart (cleared by a fill kernel)
  int32_t nu, na, nt, ne;   // product-grid axes (na = 0 for trajectory lists)
  int32_t traj_per_item;
  int32_t waves_per_block;
  int32_t grid_blocks;
  int32_t tu;               // trajectories scored together per wavefront (1, 2 or 4)
  const int32_t* perm;      // trajectory lists: [lists][n_traj] scoring order, or nullptr
};
// Scoring order of trajectory lists (n_lists lists of n_traj, their constants in tc):
// each list grouped by direction, kPermBins buckets of alpha, so that waves scoring at
// the same time follow nearby lines through the map (a counting sort; the order within
// a bucket is unspecified and changes the schedule only); perm holds indices over all
// lists (list * n_traj + trajectory).  key: n_lists * n_traj words of workspace, hist:
// n_lists * kPermBins counters.  Lists with more than kPermBinsMax counters in all are
// not reordered by the caller.
constexpr int kPermBins = 256;
constexpr int64_t kPermBinsMax = 1 << 22;
hipError_t launch_traj_perm(const TrajC* tc, int64_t n_traj, int32_t n_lists, uint32_t* key,
                            uint32_t* hist, int32_t* perm, hipStream_t st);
// Work queues of the batched search (one per XCD) and the words they occupy.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;
constexpr int kQueueWords = kQueues * kQueueStride;
hipError_t launch_search_batched(const BatchedArgs& a, hipStream_t st);

// Best (chi2, index) per segment of length seg_len; n_seg segments.
hipError_t launch_best(const double* chi2, int64_t n_seg, int64_t seg_len, double* best_chi2,
                       int64_t* best_idx, hipStream_t st);
// Top-k per segment (k <= 4096); scratch of topk_scratch_bytes(n_seg, k) bytes.
size_t topk_scratch_bytes(int64_t n_seg, int32_t k);
hipError_t launch_topk(const double* chi2, int64_t n_seg, int64_t seg_len, int32_t k,
                       double* out_chi2, int64_t* out_idx, void* scratch, int num_cu,
                       hipStream_t st);

// Expand top-k flat indices (map * n_traj + traj) into parameter rows.
hipError_t launch_candidates(const double* axes, int32_t nu, int32_t na, int32_t nt, int32_t ne,
                             const double* list, int32_t shared, int64_t n_traj, int32_t n_events,
                             int32_t n_maps, int32_t k, const int64_t* idx, double* params,
                             int32_t* event, int32_t* mapidx, hipStream_t st);

// Gradient evaluation.  When `anchor`/`pt` are given the parameters are the
// L-BFGS variables (natural = anchor mapped by pt) and the gradient is written with
// respect to pt; `active` (nullable) skips finished candidates.
struct GradArgs {
  int64_t n;
  const double* params;     // natural [n][4] (when anchor == nullptr)
  const double* anchor;     // [n][4] or nullptr
  const float* pt;          // [n][4] or nullptr
  const int32_t* active;    // [n] or nullptr
  const int32_t* event;
  const int32_t* mapidx;
  const MapC* maps;
  int32_t n_events, n_maps;  // out-of-range event / map indices give NaN outputs
  TrajC* tc;                 // [n] per-candidate constants (written by the prep kernel)
  double* tEv;               // [n] FP64 tE of each candidate
  LcView lc;
  double* chi2;
  double* grad;             // [n][4] or nullptr
  double* fs;
  double* fb;
  const int32_t* order;     // [n] the order in which candidates are evaluated, or nullptr
};
// Per-candidate constants (FP64 natural parameters -> binary32 TrajC), then the
// evaluation kernel.
hipError_t launch_cand_prep(const GradArgs& a, hipStream_t st);
hipError_t launch_chi2_grad(const GradArgs& a, hipStream_t st);
// Evaluation order of candidates [0, a.n): grouped by (map, event) (by map alone when
// n_maps x n_events exceeds kOrderBinsMax), so that candidates evaluated at the same
// time sample the same map.  Within a group the order is unspecified: it changes only
// the schedule, never a result.  key: workspace of a.n words; hist: of order_bins(a)
// counters.
constexpr int64_t kOrderBinsMax = 1 << 20;
inline int64_t order_bins(int32_t n_maps, int32_t n_events) {
  const int64_t both = (int64_t)n_maps * n_events;
  return both <= kOrderBinsMax ? both : n_maps;
}
hipError_t launch_cand_order(const GradArgs& a, uint32_t* key, uint32_t* hist, int32_t* order,
                             hipStream_t st);

struct LbfgsState {
  int64_t n;
  int32_t m;
  int32_t max_ls;
  double c1, shrink;
  const double* anchor;  // [n][4]
  float* p;              // [n][4] accepted point
  float* pt;             // [n][4] trial point
  double* f;             // [n]
  double* g;             // [n][4]
  double* d;             // [n][4]
  double* step;          // [n]
  double* S;             // [n][m][4] history pairs, oldest first
  double* Y;             // [n][m][4]
  double* R;             // [n][m]
  int32_t* nhist;        // [n]
  int32_t* nls;          // [n]
  int32_t* active;       // [n]
};
// Anchor copy, state reset and first-trial trajectory constants (a.tc, a.tEv).
hipError_t launch_refine_init(const LbfgsState& s, const GradArgs& a, const double* params,
                              double* anchor, hipStream_t st);
// One update of every active candidate from its evaluation ft [n], gt [n][4], then the
// trajectory constants of its next trial; round 0 also copies ft to chi2_init (if set).
// s.m must be at most 16.
hipError_t launch_lbfgs_update(const LbfgsState& s, const GradArgs& a, int32_t round,
                               const double* ft, const double* gt, double* chi2_init,
                               hipStream_t st);
hipError_t launch_lbfgs_finish(const LbfgsState& s, double* params, double* chi2_out,
                               hipStream_t st);

}  // namespace morse
