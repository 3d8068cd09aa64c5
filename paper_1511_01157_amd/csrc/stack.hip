// FFT convolution for finite-source map stacks on gfx950.
//
// A finite-source map is the count map convolved with the pixel weights of a source
// profile (sec. 4.1 of McDougall & Albrow 2015: point-source maps convolved with
// limb-darkened profiles of several radii).  For radii spanning tens to hundreds of
// pixels the direct stencil sum costs (2R+1)^2 products per pixel, so the wide
// profiles go through the convolution theorem instead: the count map, extended past
// its edges by its edge pixels (the clamp rule of the direct sum), is transformed once;
// each pair of profiles is packed as w1 + i w2 (both real and even, so their transforms
// are real and the products separate into the real and imaginary parts of one inverse
// transform); one inverse transform then yields two maps.  All arithmetic is FP64 and
// each output is rounded once to binary32.
//
// Transform layout.  Complex FP64 arrays [ny][nx], natural order, power-of-two sizes.
// Along x one workgroup holds a whole row in LDS and runs the Stockham passes there
// (radix 16, then 8, 4 or 2 for the remainder); along y each pass runs in global memory
// with consecutive lanes on consecutive columns, so every load and store of a wavefront
// is one contiguous 1 KiB segment.  Forward (counts): the rows of the map only (the
// padded rows above and below repeat the edge rows), each padded in x and transformed,
// keeping the columns 0 .. nx/2 (the input is real, so the other half is the conjugate
// reflection); then the columns of that half spectrum, the first pass reading each
// padded row from its map row.  Inverse (per pair of profiles): columns, the first pass
// rebuilding the full spectrum by conjugate reflection and multiplying by the pair's
// transform, the last writing only the map's rows; then those rows (fused with the
// crop, the scale and the binary32 store).  The profile transforms use full arrays.

#include "stack.h"

namespace morse {

namespace {

constexpr int kRowThreads = 256;

struct Cx {
  double re, im;
};

__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx cmul(Cx a, Cx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx ld(const double2& v) { return {v.x, v.y}; }
__device__ __forceinline__ double2 st(Cx v) { return make_double2(v.re, v.im); }

// exp(SGN 2 pi i m / 16), m = 0 .. 15
template <int SGN>
__device__ __forceinline__ Cx w16(int m) {
  constexpr double c1 = 0.92387953251128674, c2 = 0.70710678118654752, c3 = 0.38268343236508977;
  constexpr double cs[16] = {1, c1, c2, c3, 0, -c3, -c2, -c1, -1, -c1, -c2, -c3, 0, c3, c2, c1};
  constexpr double sn[16] = {0, c3, c2, c1, 1, c1, c2, c3, 0, -c3, -c2, -c1, -1, -c1, -c2, -c3};
  return {cs[m & 15], SGN * sn[m & 15]};
}

// x * (SGN i)
template <int SGN>
__device__ __forceinline__ Cx rot(Cx x) {
  return {-SGN * x.im, SGN * x.re};
}

template <int SGN>
__device__ __forceinline__ void dft2(Cx& a, Cx& b) {
  const Cx t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// in place: (x0, x1, x2, x3) -> its 4-point DFT with kernel exp(SGN 2 pi i / 4)
template <int SGN>
__device__ __forceinline__ void dft4(Cx& x0, Cx& x1, Cx& x2, Cx& x3) {
  const Cx a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = rot<SGN>(csub(x1, x3));
  x0 = cadd(a0, a2);
  x1 = cadd(a1, a3);
  x2 = csub(a0, a2);
  x3 = csub(a1, a3);
}

// R-point DFT of v (R = 2, 4, 8, 16), kernel exp(SGN 2 pi i / R).  For R = 4P the index
// splits as n = P n1 + n2, k = k1 + 4 k2: 4-point DFTs over n1, twiddles
// exp(SGN 2 pi i n2 k1 / R), then P-point DFTs over n2.
template <int R, int SGN>
__device__ __forceinline__ void dft(Cx (&v)[R]) {
  if constexpr (R == 2) {
    dft2<SGN>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<SGN>(v[0], v[1], v[2], v[3]);
  } else {
    constexpr int P = R / 4;
    Cx y[P][4];
#pragma unroll
    for (int n2 = 0; n2 < P; ++n2) {
      y[n2][0] = v[n2];
      y[n2][1] = v[P + n2];
      y[n2][2] = v[2 * P + n2];
      y[n2][3] = v[3 * P + n2];
      dft4<SGN>(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1)
        if (n2 * k1 != 0) y[n2][k1] = cmul(y[n2][k1], w16<SGN>(n2 * k1 * (16 / R)));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      if constexpr (P == 2) {
        Cx a = y[0][k1], b = y[1][k1];
        dft2<SGN>(a, b);
        v[k1] = a;
        v[k1 + 4] = b;
      } else {
        Cx a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
        dft4<SGN>(a, b, c, d);
        v[k1] = a;
        v[k1 + 4] = b;
        v[k1 + 8] = c;
        v[k1 + 12] = d;
      }
    }
  }
}

// Twiddle exp(SGN 2 pi i m / n) from the table tw[m] = exp(-2 pi i m / n).
template <int SGN>
__device__ __forceinline__ Cx twiddle(const double2* tw, int m) {
  const double2 t = tw[m];
  return {t.x, SGN == -1 ? t.y : -t.y};
}

// One Stockham pass of radix R over the n values in LDS (ns = product of the radices
// before it): butterfly j reads s[j + r n/R], twiddles by exp(SGN 2 pi i r k/(ns R))
// with k = j mod ns, and writes s[(j/ns) ns R + k + r ns].  Every value is read into
// registers before the barrier, so one buffer serves as input and output.
template <int R, int SGN>
__device__ __forceinline__ void lds_pass(double2* s, int n, int ns, const double2* tw) {
  const int j = threadIdx.x;
  const int nb = n / R;
  const bool act = j < nb;
  Cx v[R];
  int k = 0;
  if (act) {
    k = j & (ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ld(s[j + r * nb]);
    if (ns > 1) {
      const int step = n / (ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle<SGN>(tw, r * k * step));
    }
    dft<R, SGN>(v);
  }
  __syncthreads();
  if (act) {
    const int base = (j / ns) * ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) s[base + r * ns] = st(v[r]);
  }
  __syncthreads();
}

// Whole transform of the n values in s (n a power of two, n <= kRowThreads * 16).
template <int SGN>
__device__ void lds_fft(double2* s, int n, const double2* tw) {
  int ns = 1;
  while (ns < n) {
    const int rem = n / ns;
    if (rem >= 16) {
      lds_pass<16, SGN>(s, n, ns, tw);
      ns *= 16;
    } else if (rem == 8) {
      lds_pass<8, SGN>(s, n, ns, tw);
      ns *= 8;
    } else if (rem == 4) {
      lds_pass<4, SGN>(s, n, ns, tw);
      ns *= 4;
    } else {
      lds_pass<2, SGN>(s, n, ns, tw);
      ns *= 2;
    }
  }
}

// Map index of padded position p (n positions, m map pixels): p itself below
// m + (n - m)/2, p - n above, clamped to the map (edge-pixel extension).
__device__ __forceinline__ int pad_index(int p, int n, int m) {
  const int i = p < m + (n - m) / 2 ? p : p - n;
  return i < 0 ? 0 : (i > m - 1 ? m - 1 : i);
}

// Map row y (grid = my): transform of its padded row; columns 0 .. nx/2 stored (the
// rest follow by Hermitian symmetry, the row being real), out[my][nx/2 + 1].
__global__ __launch_bounds__(kRowThreads) void k_fft_rows_counts(FftGrid g, const uint32_t* counts,
                                                                 int32_t mx, int32_t my,
                                                                 double2* out) {
  __shared__ double2 s[kFftMaxN];
  const int y = blockIdx.x;
  const uint32_t* row = counts + (size_t)y * mx;
  for (int x = threadIdx.x; x < g.nx; x += kRowThreads)
    s[x] = make_double2((double)row[pad_index(x, g.nx, mx)], 0.0);
  __syncthreads();
  lds_fft<-1>(s, g.nx, g.tw_x);
  const int h = g.nx / 2 + 1;
  double2* o = out + (size_t)y * h;
  for (int x = threadIdx.x; x < h; x += kRowThreads) o[x] = s[x];
}

__device__ __forceinline__ double quad_weight(const double* q, int rx, int ry, int a, int b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  return (q && a <= rx && b <= ry) ? q[(size_t)b * (rx + 1) + a] : 0.0;
}

__global__ __launch_bounds__(kRowThreads) void k_fft_rows_taps(FftGrid g, const double* q1,
                                                               int32_t r1x, int32_t r1y,
                                                               const double* q2, int32_t r2x,
                                                               int32_t r2y, double2* out) {
  __shared__ double2 s[kFftMaxN];
  const int y = blockIdx.x;
  const int b = y < g.ny / 2 ? y : y - g.ny;
  for (int x = threadIdx.x; x < g.nx; x += kRowThreads) {
    const int a = x < g.nx / 2 ? x : x - g.nx;
    s[x] = make_double2(quad_weight(q1, r1x, r1y, a, b), quad_weight(q2, r2x, r2y, a, b));
  }
  __syncthreads();
  lds_fft<-1>(s, g.nx, g.tw_x);
  double2* o = out + (size_t)y * g.nx;
  for (int x = threadIdx.x; x < g.nx; x += kRowThreads) o[x] = s[x];
}

__global__ __launch_bounds__(kRowThreads) void k_fft_rows_store(FftGrid g, const double2* in,
                                                                int32_t mx, int32_t my,
                                                                double scale, float* map1,
                                                                float* map2) {
  __shared__ double2 s[kFftMaxN];
  const int y = blockIdx.x;  // padded row y < my is map row y
  const double2* row = in + (size_t)y * g.nx;
  for (int x = threadIdx.x; x < g.nx; x += kRowThreads) s[x] = row[x];
  __syncthreads();
  lds_fft<1>(s, g.nx, g.tw_x);
  float* o1 = map1 + (size_t)y * mx;
  float* o2 = map2 ? map2 + (size_t)y * mx : nullptr;
  for (int x = threadIdx.x; x < mx; x += kRowThreads) {
    const double2 v = s[x];
    o1[x] = (float)(v.x * scale);
    if (o2) o2[x] = (float)(v.y * scale);
  }
}

// One Stockham pass along y for columns 0 .. ncols - 1 (the row pass's indexing with
// rows in place of LDS slots); thread t takes column t mod ncols and butterfly t / ncols.
// The first pass of a transform may read a compact padded input (row -> its map row)
// or a Hermitian half spectrum (columns beyond herm_cols by conjugate reflection) and
// multiply by a spectral product; the last may skip rows the caller does not read.
struct ColPassArgs {
  int32_t ncols, in_stride, out_stride, ns;
  int32_t map_rows, herm_cols, out_rows;
};

template <int R, int SGN, bool MUL>
__global__ __launch_bounds__(256) void k_fft_col_pass(FftGrid g, ColPassArgs c, const double2* in,
                                                      double2* out, const double2* mul) {
  const int n = g.ny;
  const int nb = n / R;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * c.ncols) return;
  const int x = (int)(t % c.ncols);
  const int j = (int)(t / c.ncols);
  Cx v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = j + r * nb;
    if (c.map_rows > 0) {
      v[r] = ld(in[(size_t)pad_index(row, n, c.map_rows) * c.in_stride + x]);
    } else if (c.herm_cols > 0 && x >= c.herm_cols) {
      const Cx e = ld(in[(size_t)((n - row) & (n - 1)) * c.in_stride + (g.nx - x)]);
      v[r] = {e.re, -e.im};
    } else {
      v[r] = ld(in[(size_t)row * c.in_stride + x]);
    }
    if (MUL) v[r] = cmul(v[r], ld(mul[(size_t)row * g.nx + x]));
  }
  const int k = j & (c.ns - 1);
  if (c.ns > 1) {
    const int step = n / (c.ns * R);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle<SGN>(g.tw_y, r * k * step));
  }
  dft<R, SGN>(v);
  const int base = (j / c.ns) * c.ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int orow = base + r * c.ns;
    if (orow < c.out_rows) out[(size_t)orow * c.out_stride + x] = st(v[r]);
  }
}

template <int SGN, bool MUL>
hipError_t col_pass(const FftGrid& g, int R, const ColPassArgs& c, const double2* in, double2* out,
                    const double2* mul, hipStream_t st) {
  const int64_t threads = (int64_t)(g.ny / R) * c.ncols;
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (R) {
    case 16: hipLaunchKernelGGL((k_fft_col_pass<16, SGN, MUL>), grid, dim3(256), 0, st, g, c, in, out, mul); break;
    case 8: hipLaunchKernelGGL((k_fft_col_pass<8, SGN, MUL>), grid, dim3(256), 0, st, g, c, in, out, mul); break;
    case 4: hipLaunchKernelGGL((k_fft_col_pass<4, SGN, MUL>), grid, dim3(256), 0, st, g, c, in, out, mul); break;
    default: hipLaunchKernelGGL((k_fft_col_pass<2, SGN, MUL>), grid, dim3(256), 0, st, g, c, in, out, mul); break;
  }
  return hipGetLastError();
}

bool valid(const FftGrid& g) {
  auto pow2 = [](int32_t n) { return n >= 2 && n <= kFftMaxN && (n & (n - 1)) == 0; };
  return pow2(g.nx) && pow2(g.ny) && g.tw_x && g.tw_y;
}

}  // namespace

hipError_t launch_fft_rows_counts(const FftGrid& g, const uint32_t* counts, int32_t mx, int32_t my,
                                  double2* out, hipStream_t st) {
  if (!valid(g) || mx < 1 || my < 1 || mx > g.nx || my > g.ny) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fft_rows_counts, dim3((unsigned)my), dim3(kRowThreads), 0, st, g, counts, mx,
                     my, out);
  return hipGetLastError();
}

hipError_t launch_fft_rows_taps(const FftGrid& g, const double* q1, int32_t r1x, int32_t r1y,
                                const double* q2, int32_t r2x, int32_t r2y, double2* out,
                                hipStream_t st) {
  if (!valid(g) || !q1 || 2 * r1x + 1 > g.nx || 2 * r1y + 1 > g.ny ||
      (q2 && (2 * r2x + 1 > g.nx || 2 * r2y + 1 > g.ny)))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fft_rows_taps, dim3((unsigned)g.ny), dim3(kRowThreads), 0, st, g, q1, r1x,
                     r1y, q2, r2x, r2y, out);
  return hipGetLastError();
}

hipError_t launch_fft_cols(const FftGrid& g, const ColTransform& ct, const double2* src, double2* a,
                           double2* b, double2** result, hipStream_t st) {
  if (!valid(g) || !src || !a || !b || a == b || (ct.sign != 1 && ct.sign != -1) || ct.ncols < 1 ||
      ct.ncols > g.nx || ct.src_stride < (ct.herm_cols > 0 ? ct.herm_cols : ct.ncols) ||
      ct.stride < ct.ncols || ct.map_rows < 0 ||
      ct.map_rows > g.ny || ct.herm_cols < 0 || ct.herm_cols > g.nx / 2 + 1 ||
      (ct.herm_cols > 0 && ct.ncols != g.nx) || ct.last_rows < 1 || ct.last_rows > g.ny)
    return hipErrorInvalidValue;
  const double2* cur = src;
  double2* dst = (src == a) ? b : a;
  ColPassArgs c{ct.ncols, ct.src_stride, ct.stride, 1, ct.map_rows, ct.herm_cols, g.ny};
  bool first = true;
  while (c.ns < g.ny) {
    const int R = (g.ny / c.ns >= 16) ? 16 : g.ny / c.ns;
    if (c.ns * R == g.ny) c.out_rows = ct.last_rows;  // the last pass
    const double2* m = first ? ct.mul : nullptr;
    hipError_t e;
    if (ct.sign < 0)
      e = m ? col_pass<-1, true>(g, R, c, cur, dst, m, st) : col_pass<-1, false>(g, R, c, cur, dst, m, st);
    else
      e = m ? col_pass<1, true>(g, R, c, cur, dst, m, st) : col_pass<1, false>(g, R, c, cur, dst, m, st);
    if (e != hipSuccess) return e;
    cur = dst;
    dst = (dst == a) ? b : a;
    c.ns *= R;
    first = false;
    c.in_stride = ct.stride;  // passes after the first read the work buffers
    c.map_rows = 0;
    c.herm_cols = 0;
  }
  *result = const_cast<double2*>(cur);
  return hipSuccess;
}

hipError_t launch_fft_rows_store(const FftGrid& g, const double2* in, int32_t mx, int32_t my,
                                 double scale, float* map1, float* map2, hipStream_t st) {
  if (!valid(g) || !in || !map1 || mx < 1 || my < 1 || mx > g.nx || my > g.ny)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fft_rows_store, dim3((unsigned)my), dim3(kRowThreads), 0, st, g, in, mx, my,
                     scale, map1, map2);
  return hipGetLastError();
}

}  // namespace morse
