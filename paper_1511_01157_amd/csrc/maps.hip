// Map build on gfx950: inverse ray shooting into LDS-privatised uint32 histogram
// tiles merged with global atomics, then normalisation + uniform-disk convolution.
//
// Method: ray-shooting magnification maps (the family cited in sec. 3 of McDougall &
// Albrow 2015) of the binary-lens equation Eq. 2 with the lens placement of sec. 4.1;
// finite-source maps by convolution with the source profile (sec. 4.1).
//
// Ray kernel layout.  A 256-thread workgroup owns a 128 x 64 tile of the image-plane
// lattice (32 rays per thread).  Rays are generated from their indices (no input
// arrays).  Thread (tx, ty) of a 16 x 16 arrangement takes rays x0 + tx + 16a,
// y0 + ty + 16b, so the 64 lanes of a wave at one (a, b) are spread over a 16 x 4
// patch of rays, i.e. over several source pixels, which keeps LDS atomics of one
// instruction off a single address.  Pass 1 computes every ray's bin and the
// workgroup's bounding box of in-window bins.  If the box fits in the LDS tile
// (8192 bins) the rays are counted with LDS atomics and the non-zero bins merged
// with one global atomic each; otherwise (tiles straddling a lens, whose rays scatter
// over the whole source plane) each ray goes to a global atomic directly.  Integer
// addition is order-free, so the counts are bit-identical whatever the schedule.
//
// Mirror pairs.  With both lenses on the x axis, a lattice centred on y = 0 with an
// even row count and a window centred on y = 0, the ray of row ny - 1 - j is the
// mirror image of the ray of row j: its y is exactly -y, and since binary32 rounding
// commutes with negation every step of Eq. 2 gives exactly the same x and the negated
// y, so its bin is (bx, 2h - 1 - by) by the symmetric bin rule (h = my / 2), unless
// its y offset in the window is +-0, when both rays fall in row h.  Rows that have
// their mirror row in the same call are then shot once, from the upper half, and each
// binned ray is counted in both bins (the +-0 rays twice in their own bin); the ray
// statistics count every shot ray twice.

#include <algorithm>

#include "internal.h"

#include <climits>

namespace morse {

namespace {

constexpr int RS_TX = 128;
constexpr int RS_TY = 64;
constexpr int RS_THREADS = 256;
constexpr int RS_A = RS_TX / 16;  // rays per thread along x
constexpr int RS_B = RS_TY / 16;  // rays per thread along y
constexpr int RS_CAP = 8192;      // LDS histogram bins (32 KiB)

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, size_t n, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Quad packing of one map per blockIdx.y (layout in MapC); cells beyond the map
// (tile padding) are zero and never sampled.
__global__ void k_quad_pack(const MapC* __restrict__ maps) {
  const MapC m = maps[blockIdx.y];
  const uint64_t nq = (uint64_t)m.tiles_x * m.tiles_y * 8;
  Quad* out = const_cast<Quad*>(m.quad);
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nq;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t tile = q >> 3;
    const uint32_t r = (uint32_t)(q & 7);
    const uint64_t i = (tile % m.tiles_x) * 4 + (r >> 1);
    const uint64_t j = (tile / m.tiles_x) * 2 + (r & 1u);
    Quad v = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i + 1 < (uint64_t)m.mx && j + 1 < (uint64_t)m.my) {
      const float* row = m.map + j * (uint64_t)m.mx + i;
      v.v00 = row[0];
      v.v10 = row[1];
      v.v01 = row[m.mx];
      v.v11 = row[m.mx + 1];
    }
    out[q] = v;
  }
}

// Symmetric bin rule: v >= 0 (also -0) -> m/2 + floor(v) if v < m/2;
// v < 0 -> m/2 - 1 - floor(-v) if -v < m/2.  floor(|v|) serves both branches.
__device__ __forceinline__ bool bin1(float v, int32_t m, int32_t& out) {
  float av = fabsf(v);
  int32_t h = m >> 1;
  int32_t f = (int32_t)floorf(fminf(av, (float)h));  // clamp keeps the cast in range
  out = (v >= 0.0f) ? h + f : h - 1 - f;
  return av < (float)h;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <bool kMirror>
__global__ __launch_bounds__(RS_THREADS) void k_rayshoot(RayParams p, uint32_t* __restrict__ counts,
                                                         unsigned long long* __restrict__ stats) {
  __shared__ uint32_t hist[RS_CAP];
  __shared__ int s_box[4][4];

  const int tid = threadIdx.x;
  const int tx = tid & 15;
  const int ty = tid >> 4;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int x0 = blockIdx.x * RS_TX;
  const int y0 = p.row0 + blockIdx.y * RS_TY;

  // packed bin (by << 16 | bx), -1 when the ray is not binned
  int bins[RS_A * RS_B];
  int bxmin = INT_MAX, bxmax = -1, bymin = INT_MAX, bymax = -1;
  uint32_t n_out = 0, n_nf = 0, n_zero = 0;

#pragma unroll
  for (int b = 0; b < RS_B; ++b) {
    const int j = y0 + ty + 16 * b;
    const float gy = (float)(j - (p.ny >> 1)) + 0.5f;
    const float y = p.cy + gy * p.hy;
    const float yy = y * y;
#pragma unroll
    for (int a = 0; a < RS_A; ++a) {
      const int i = x0 + tx + 16 * a;
      int bin = -1;
      if (i < p.nx && j < p.row1) {
        const float gx = (float)(i - (p.nx >> 1)) + 0.5f;
        const float x = p.cx + gx * p.hx;
        const float d1 = x - p.x1;
        const float d2 = x - p.x2;
        const float r1 = d1 * d1 + yy;
        const float r2 = d2 * d2 + yy;
        const float a1 = p.m1 / r1;
        const float a2 = p.m2 / r2;
        const float zx = (x - a1 * d1) - a2 * d2;
        const float zy = (y - a1 * y) - a2 * y;
        const float vx = (zx - p.sx) * p.kx;
        const float vy = (zy - p.sy) * p.ky;
        if (!(isfinite(vx) && isfinite(vy))) {
          ++n_nf;
        } else {
          int32_t bx, by;
          const bool inx = bin1(vx, p.mx, bx);
          const bool iny = bin1(vy, p.my, by);
          if (inx && iny && kMirror && vy == 0.0f) {
            // the ray and its mirror share the bin (bx, h)
            atomicAdd(&counts[(size_t)by * (size_t)p.mx + (size_t)bx], 2u);
            ++n_zero;
          } else if (inx && iny) {
            bin = (by << 16) | bx;
            n_zero += (vy == 0.0f) ? 1u : 0u;
            bxmin = min(bxmin, bx);
            bxmax = max(bxmax, bx);
            bymin = min(bymin, by);
            bymax = max(bymax, by);
          } else {
            ++n_out;
          }
        }
      }
      bins[b * RS_A + a] = bin;
    }
  }

  // ray statistics: one 64-bit atomic per wave and counter, only when non-zero
  constexpr uint32_t kRays = kMirror ? 2u : 1u;  // rays each shot ray stands for
  n_out = wave_sum_u32(n_out) * kRays;
  n_nf = wave_sum_u32(n_nf) * kRays;
  n_zero = wave_sum_u32(n_zero) * kRays;
  if (lane == 0 && stats) {
    if (n_out) atomicAdd(&stats[0], (unsigned long long)n_out);
    if (n_nf) atomicAdd(&stats[1], (unsigned long long)n_nf);
    if (n_zero) atomicAdd(&stats[2], (unsigned long long)n_zero);
  }

  // workgroup bounding box of binned rays
  bxmin = wave_min(bxmin);
  bxmax = wave_max(bxmax);
  bymin = wave_min(bymin);
  bymax = wave_max(bymax);
  if (lane == 0) {
    s_box[wave][0] = bxmin;
    s_box[wave][1] = bxmax;
    s_box[wave][2] = bymin;
    s_box[wave][3] = bymax;
  }
  __syncthreads();
  bxmin = min(min(s_box[0][0], s_box[1][0]), min(s_box[2][0], s_box[3][0]));
  bxmax = max(max(s_box[0][1], s_box[1][1]), max(s_box[2][1], s_box[3][1]));
  bymin = min(min(s_box[0][2], s_box[1][2]), min(s_box[2][2], s_box[3][2]));
  bymax = max(max(s_box[0][3], s_box[1][3]), max(s_box[2][3], s_box[3][3]));
  if (bxmax < 0) return;  // no ray of this tile landed in the window

  const int pitch = bxmax - bxmin + 1;
  const int rows = bymax - bymin + 1;
  const int area = pitch * rows;
  if (area <= RS_CAP) {
    for (int k = tid; k < area; k += RS_THREADS) hist[k] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS_A * RS_B; ++k) {
      const int bin = bins[k];
      if (bin >= 0) {
        const int bx = bin & 0xffff;
        const int by = bin >> 16;
        atomicAdd(&hist[(by - bymin) * pitch + (bx - bxmin)], 1u);
      }
    }
    __syncthreads();
    const int top = 2 * (p.my >> 1) - 1;  // mirror row of by is top - by
    for (int k = tid; k < area; k += RS_THREADS) {
      const uint32_t v = hist[k];
      if (v) {
        const int r = k / pitch;
        const int c = k - r * pitch;
        atomicAdd(&counts[(size_t)(bymin + r) * (size_t)p.mx + (size_t)(bxmin + c)], v);
        if (kMirror)
          atomicAdd(&counts[(size_t)(top - (bymin + r)) * (size_t)p.mx + (size_t)(bxmin + c)], v);
      }
    }
  } else {
    const int top = 2 * (p.my >> 1) - 1;
#pragma unroll
    for (int k = 0; k < RS_A * RS_B; ++k) {
      const int bin = bins[k];
      if (bin >= 0) {
        const int bx = bin & 0xffff;
        const int by = bin >> 16;
        atomicAdd(&counts[(size_t)by * (size_t)p.mx + (size_t)bx], 1u);
        if (kMirror) atomicAdd(&counts[(size_t)(top - by) * (size_t)p.mx + (size_t)bx], 1u);
      }
    }
  }
}

// Normalise + convolve.  Taps are row-major over the stencil with the zero taps dropped
// on the host; neighbours clamp to the edge; acc accumulates the terms w[k] * count in
// tap order in binary32 (the first term alone, then one addition per tap) and
// A = acc * scale.  The kernels also reduce the largest count of the map (one atomic
// per workgroup).  Three forms of the same arithmetic:
//   * one tap at offset (0, 0) (a point source): elementwise, four pixels per thread
//     with 16-byte loads and stores;
//   * a stencil of half-width at most kNcHalo: a workgroup stages a 64 x 32 output tile
//     plus halo in LDS (sized to the stencil; counts converted to binary32 there, the
//     conversion every term applies), then each wave sweeps whole 64-pixel rows, so LDS
//     reads are consecutive and stores 256 B per row; each wave issues all its staging
//     loads (whole tile rows) before the first LDS store.  The tap builders cap the
//     half-width at 15 pixels;
//   * a stencil of reach at most one pixel (3 x 3) on a map whose width is a multiple
//     of 4 with 16-byte aligned buffers: no LDS.  A wavefront takes kR1Cols = 256
//     columns (four per lane, 16-byte loads and stores) and kR1Rows rows, loading the
//     rows y0 - 1 .. y0 + kR1Rows (clamped) and, by scalar loads, the column on each
//     side of its 256; a lane's outer neighbours come from the adjacent lanes by DPP
//     wavefront shifts, the wavefront's outer lanes taking the side columns.  The terms are added in raster order over the 3 x 3 neighbourhood with a
//     zero weight where the tap list has no tap: that is the tap order, and a zero term
//     (0 * count = +0) leaves a sum of non-negative terms unchanged, so the arithmetic
//     is that of the tap list.
constexpr int kNcTw = 64, kNcTh = 32, kNcHalo = 16;
constexpr int kR1Cols = 256, kR1Rows = 8;

__device__ __forceinline__ void nc_block_max(uint32_t cmax, uint32_t* maxc) {
  __shared__ uint32_t s_max[4];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, o, kWave));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = cmax;
  __syncthreads();
  if (threadIdx.x == 0 && maxc) atomicMax(maxc, max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3])));
}

__global__ __launch_bounds__(256) void k_normalize_point(const uint32_t* __restrict__ counts,
                                                         float* __restrict__ map, int64_t npx,
                                                         bool vec4, const float* __restrict__ w,
                                                         float scale, uint32_t* __restrict__ maxc) {
  const float w0 = w[0];
  uint32_t cmax = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (vec4) {
    const uint4* c4 = reinterpret_cast<const uint4*>(counts);
    float4* m4 = reinterpret_cast<float4*>(map);
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < npx / 4; v += stride) {
      const uint4 c = c4[v];
      cmax = max(max(cmax, max(c.x, c.y)), max(c.z, c.w));
      m4[v] = make_float4((w0 * (float)c.x) * scale, (w0 * (float)c.y) * scale,
                          (w0 * (float)c.z) * scale, (w0 * (float)c.w) * scale);
    }
  } else {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < npx; v += stride) {
      const uint32_t c = counts[v];
      cmax = max(cmax, c);
      map[v] = (w0 * (float)c) * scale;
    }
  }
  nc_block_max(cmax, maxc);
}

__global__ __launch_bounds__(256) void k_normalize_convolve_lds(
    const uint32_t* __restrict__ counts, float* __restrict__ map, int32_t mx, int32_t my,
    const float* __restrict__ w, const int32_t* __restrict__ off, int32_t ntaps, int32_t rx,
    int32_t ry, float scale, uint32_t* __restrict__ maxc) {
  extern __shared__ float tile[];  // (kNcTw + 2 rx) x (kNcTh + 2 ry)
  const int x0 = blockIdx.x * kNcTw, y0 = blockIdx.y * kNcTh;
  const int lw = kNcTw + 2 * rx, lh = kNcTh + 2 * ry;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // staging: wave w takes tile rows w, w + 4, ...; lane l the columns l and 64 + l; all
  // loads are issued before the first LDS store
  constexpr int kRowsPerWave = (kNcTh + 2 * kNcHalo + 3) / 4;
  uint32_t va[kRowsPerWave], vb[kRowsPerWave];
  const int gxa = min(max(x0 - rx + lane, 0), mx - 1), gxb = min(max(x0 - rx + 64 + lane, 0), mx - 1);
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const int ly = wave + 4 * r;
    va[r] = vb[r] = 0u;
    if (ly < lh) {  // uniform per wave
      const uint32_t* row = counts + (size_t)min(max(y0 - ry + ly, 0), my - 1) * mx;
      va[r] = row[gxa];
      if (lane < lw - 64) vb[r] = row[gxb];
    }
  }
  uint32_t cmax = 0;
  const bool own_a = lane >= rx && x0 - rx + lane < mx;  // own columns: [rx, rx + 64)
  const bool own_b = lane < rx && x0 - rx + 64 + lane < mx;  // and [64, 64 + rx)
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const int ly = wave + 4 * r;
    if (ly < lh) {
      tile[ly * lw + lane] = (float)va[r];
      if (lane < lw - 64) tile[ly * lw + 64 + lane] = (float)vb[r];
      if (ly >= ry && ly < ry + kNcTh && y0 - ry + ly < my) {
        if (own_a) cmax = max(cmax, va[r]);
        if (own_b) cmax = max(cmax, vb[r]);
      }
    }
  }
  __syncthreads();
  constexpr int kRows = kNcTh / 4;
  float acc[kRows];
  for (int k = 0; k < ntaps; ++k) {
    const float wk = w[k];
    const int base = (wave + ry + off[2 * k + 1]) * lw + lane + rx + off[2 * k];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const float term = wk * tile[base + 4 * r * lw];
      acc[r] = (k == 0) ? term : acc[r] + term;
    }
  }
  const int gx = x0 + lane;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int gy = y0 + wave + 4 * r;
    if (gx < mx && gy < my) map[(size_t)gy * mx + gx] = acc[r] * scale;
  }
  nc_block_max(cmax, maxc);
}

// v of lane l - 1 (lane 0 takes lo) and of lane l + 1 (lane 63 takes hi), by DPP
// wavefront shifts.
__device__ __forceinline__ float from_lane_below(float v, float lo) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(lo), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_lane_above(float v, float hi) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(hi), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__global__ __launch_bounds__(256) void k_normalize_convolve_r1(
    const uint32_t* __restrict__ counts, float* __restrict__ map, int32_t mx, int32_t my,
    const float* __restrict__ w, const int32_t* __restrict__ off, int32_t ntaps, float scale,
    uint32_t* __restrict__ maxc) {
  const int lane = threadIdx.x & (kWave - 1);
  const int ncx = (mx + kR1Cols - 1) / kR1Cols;
  // the wave's index, read from the first lane so that everything derived from it (tile
  // origin, row offsets, the neighbouring columns' loads) stays in scalar registers;
  // 32-bit arithmetic: the launcher admits maps below 2^30 pixels
  const int item = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = item % ncx * kR1Cols;
  const int y0 = item / ncx * kR1Rows;
  uint32_t cmax = 0;
  if (y0 < my) {  // uniform per wave (the last workgroup's waves may lie past the map)
    // the 3 x 3 weights in raster order (uniform), zero where there is no tap
    float W[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) W[i] = 0.0f;
    for (int k = 0; k < ntaps; ++k) {
      const int i = (off[2 * k + 1] + 1) * 3 + off[2 * k] + 1;
      const float wk = w[k];
#pragma unroll
      for (int j = 0; j < 9; ++j) W[j] = j == i ? wk : W[j];
    }
    const int xq = x0 + 4 * lane;  // the lane's four columns xq .. xq + 3
    const bool own = xq < mx;      // mx % 4 == 0: a quad lies wholly inside or outside
    const bool has_right = xq + 4 < mx;
    const uint32_t qx = (uint32_t)min(xq, mx - 4);
    // the columns beside the wavefront's 256, clamped to the map (uniform: scalar loads)
    const uint32_t hl = (uint32_t)max(x0 - 1, 0), hr = (uint32_t)min(x0 + kR1Cols, mx - 1);
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 q[kR1Rows + 2];  // all the rows' loads in flight before the first use
    uint32_t ql[kR1Rows + 2], qr[kR1Rows + 2];
#pragma unroll
    for (int r = 0; r < kR1Rows + 2; ++r) {
      const uint32_t row = (uint32_t)min(max(y0 - 1 + r, 0), my - 1) * (uint32_t)mx;
      q[r] = ldg(reinterpret_cast<const u4*>(counts), (row + qx) >> 2);
      ql[r] = counts[row + hl];
      qr[r] = counts[row + hr];
    }
    // per row: the lane's four values and their outer neighbours (the left one of column
    // 0 is column 0 itself through the clamped load; the right one of column mx - 1 is
    // column mx - 1 itself)
    float V[kR1Rows + 2][6];
#pragma unroll
    for (int r = 0; r < kR1Rows + 2; ++r) {
      V[r][1] = (float)q[r].x;
      V[r][2] = (float)q[r].y;
      V[r][3] = (float)q[r].z;
      V[r][4] = (float)q[r].w;
      V[r][0] = from_lane_below(V[r][4], (float)ql[r]);
      const float rn = from_lane_above(V[r][1], (float)qr[r]);
      V[r][5] = has_right ? rn : V[r][4];
    }
#pragma unroll
    for (int r = 0; r < kR1Rows; ++r) {
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {  // column xq + j: values V[.][j .. j + 2]
        float acc = W[0] * V[r][j];
        acc = acc + W[1] * V[r][j + 1];
        acc = acc + W[2] * V[r][j + 2];
        acc = acc + W[3] * V[r + 1][j];
        acc = acc + W[4] * V[r + 1][j + 1];
        acc = acc + W[5] * V[r + 1][j + 2];
        acc = acc + W[6] * V[r + 2][j];
        acc = acc + W[7] * V[r + 2][j + 1];
        acc = acc + W[8] * V[r + 2][j + 2];
        o[j] = acc * scale;
      }
      const int y = y0 + r;
      if (own && y < my) {
        reinterpret_cast<float4*>(map)[((uint32_t)y * (uint32_t)mx + (uint32_t)xq) >> 2] =
            make_float4(o[0], o[1], o[2], o[3]);
        const u4 c = q[r + 1];
        cmax = max(cmax, max(max(c.x, c.y), max(c.z, c.w)));
      }
    }
  }
  nc_block_max(cmax, maxc);
}

// Exclusive prefix sum of nb counters in place by one 1024-lane workgroup: each lane
// sums a contiguous chunk, a Hillis-Steele scan over the 1024 chunk sums, then each
// lane rewrites its chunk.
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* v, int64_t nb) {
  __shared__ uint32_t part[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
  uint32_t sum = 0;
  for (int64_t b = b0; b < b1; ++b) sum += v[b];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t h = v[b];
    v[b] = run;
    run += h;
  }
}

__global__ void k_bucket_count(const uint32_t* __restrict__ key, int64_t n, uint32_t* hist) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[key[i]], 1u);
}

__global__ void k_bucket_scatter(const uint32_t* __restrict__ key, int64_t n, uint32_t* cursor,
                                 int32_t* order) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    order[atomicAdd(&cursor[key[i]], 1u)] = (int32_t)i;
}

}  // namespace

hipError_t launch_bucket_order(const uint32_t* key, int64_t n, int32_t nbins, uint32_t* hist,
                               int32_t* order, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > INT32_MAX || nbins <= 0) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32(hist, (size_t)nbins, 0u, st);
  if (e != hipSuccess) return e;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)blocks), dim3(256), 0, st, key, n, hist);
  e = launch_scan_u32(hist, nbins, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bucket_scatter, dim3((unsigned)blocks), dim3(256), 0, st, key, n, hist, order);
  return hipGetLastError();
}

hipError_t launch_scan_u32(uint32_t* v, int64_t nb, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, v, nb);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_quad_pack(const MapC* maps, const MapC* h_maps, int32_t n_maps, hipStream_t st) {
  if (n_maps <= 0) return hipSuccess;
  uint64_t most = 0;
  for (int32_t k = 0; k < n_maps; ++k)
    most = std::max<uint64_t>(most, (uint64_t)h_maps[k].tiles_x * h_maps[k].tiles_y * 8);
  uint64_t blocks = (most + 255) / 256;
  if (blocks > 65536) blocks = 65536;  // grid-stride beyond
  hipLaunchKernelGGL(k_quad_pack, dim3((unsigned)blocks, (unsigned)n_maps), dim3(256), 0, st, maps);
  return hipGetLastError();
}


namespace {

// Rows [row0, row1) of p, each ray shot once (kMirror false) or, for rows of the upper
// half whose mirror rows are part of the call, once for the pair (kMirror true).
template <bool kMirror>
hipError_t shoot_rows(RayParams p, int32_t row0, int32_t row1, uint32_t* counts,
                      unsigned long long* stats, hipStream_t st) {
  const int rows = row1 - row0;
  if (rows <= 0) return hipSuccess;
  p.row0 = row0;
  p.row1 = row1;
  dim3 grid((p.nx + RS_TX - 1) / RS_TX, (rows + RS_TY - 1) / RS_TY);
  hipLaunchKernelGGL(k_rayshoot<kMirror>, grid, dim3(RS_THREADS), 0, st, p, counts, stats);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rayshoot(const RayParams& p, uint32_t* counts, unsigned long long* stats,
                           hipStream_t st) {
  if (p.row1 <= p.row0) return hipSuccess;
  // Mirror pairs need a lattice and a window centred on y = 0 and an even row count;
  // the rows paired inside [row0, row1) form [a, b) with a + b = ny.
  const int32_t a = std::max(p.row0, p.ny - p.row1), b = std::min(p.row1, p.ny - p.row0);
  if (!(p.cy == 0.0f && p.sy == 0.0f && (p.ny & 1) == 0 && a < b))
    return shoot_rows<false>(p, p.row0, p.row1, counts, stats, st);
  hipError_t e = shoot_rows<true>(p, p.ny / 2, b, counts, stats, st);
  if (e == hipSuccess) e = shoot_rows<false>(p, p.row0, a, counts, stats, st);
  if (e == hipSuccess) e = shoot_rows<false>(p, b, p.row1, counts, stats, st);
  return e;
}

hipError_t launch_normalize_convolve(const uint32_t* counts, float* map, int32_t mx, int32_t my,
                                     const float* d_w, const int32_t* d_off, int32_t ntaps,
                                     int32_t rx, int32_t ry, float scale, uint32_t* d_maxc,
                                     hipStream_t st) {
  if (mx <= 0 || my <= 0 || ntaps < 1 || rx < 0 || ry < 0) return hipErrorInvalidValue;
  if (rx == 0 && ry == 0) {
    if (ntaps != 1) return hipErrorInvalidValue;  // only the tap (0, 0) has no reach
    const int64_t npx = (int64_t)mx * my;
    const bool vec4 = npx % 4 == 0 && ((uintptr_t)counts % 16) == 0 && ((uintptr_t)map % 16) == 0;
    int64_t blocks = ((vec4 ? npx / 4 : npx) + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_normalize_point, dim3((unsigned)blocks), dim3(256), 0, st, counts, map, npx,
                       vec4, d_w, scale, d_maxc);
  } else if (rx <= 1 && ry <= 1 && (int64_t)mx * my < ((int64_t)1 << 30) && mx % 4 == 0 &&
             ((uintptr_t)counts % 16) == 0 && ((uintptr_t)map % 16) == 0) {
    if (ntaps > 9) return hipErrorInvalidValue;
    const int64_t waves = (int64_t)((mx + kR1Cols - 1) / kR1Cols) * ((my + kR1Rows - 1) / kR1Rows);
    hipLaunchKernelGGL(k_normalize_convolve_r1, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st,
                       counts, map, mx, my, d_w, d_off, ntaps, scale, d_maxc);
  } else {
    if (rx > kNcHalo || ry > kNcHalo) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (kNcTw + 2 * rx) * (kNcTh + 2 * ry);
    dim3 grid((mx + kNcTw - 1) / kNcTw, (my + kNcTh - 1) / kNcTh);
    hipLaunchKernelGGL(k_normalize_convolve_lds, grid, dim3(256), lds, st, counts, map, mx, my, d_w,
                       d_off, ntaps, rx, ry, scale, d_maxc);
  }
  return hipGetLastError();
}

}  // namespace morse
