// Launchers of the FFT convolution kernels (stack.hip) that api_maps.hip uses for
// finite-source map stacks with stencils too wide for the direct binary32 sum.  Not
// part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace morse {

// Padded transform sizes are powers of two up to 4096 per axis, so that one row of
// FP64 complex values (64 KiB) fits in a workgroup's LDS.
constexpr int kFftMaxN = 4096;

struct FftGrid {
  int32_t nx, ny;       // padded sizes, powers of two in [2, kFftMaxN]
  const double2* tw_x;  // tw_x[m] = exp(-2 pi i m / nx), m < nx
  const double2* tw_y;  // tw_y[m] = exp(-2 pi i m / ny), m < ny
};

// Forward transform along x of the padded rows of the map rows of counts[my][mx]
// (padded position p takes map index p below m + (n - m)/2 and p - n above, clamped to
// [0, m - 1]: the edge-pixel extension), columns 0 .. nx/2 kept: out[my][nx/2 + 1].
hipError_t launch_fft_rows_counts(const FftGrid& g, const uint32_t* counts, int32_t mx, int32_t my,
                                  double2* out, hipStream_t st);

// Forward transform along x of the wrap-placed weight pair w1 + i w2: offset (a, b) sits
// at position (a mod nx, b mod ny); each weight table is one quadrant q[b][a] for
// 0 <= a <= rx, 0 <= b <= ry (the weights are even in a and in b).  q2 may be null.
hipError_t launch_fft_rows_taps(const FftGrid& g, const double* q1, int32_t r1x, int32_t r1y,
                                const double* q2, int32_t r2x, int32_t r2y, double2* out,
                                hipStream_t st);

// Transform along y of columns 0 .. ncols - 1, sign -1 (forward) or +1 (inverse,
// unscaled), as a sequence of passes that alternate between the work buffers `a` and
// `b` (row pitch `stride`), starting from `src` (row pitch src_stride; left unchanged,
// and distinct from a and b).  First-pass options: map_rows > 0 reads padded row y from
// src row pad(y) of a compact [map_rows] input; herm_cols > 0 reads a Hermitian half
// spectrum of that width (column x >= herm_cols = conj of row (ny - y) mod ny, column
// nx - x; needs ncols = nx); mul multiplies every input element by mul[y][x] ([ny][nx]).
// The last pass writes rows below last_rows only.  *result = the buffer with the output.
struct ColTransform {
  int sign;
  int32_t ncols, src_stride, stride;
  int32_t map_rows, herm_cols;
  const double2* mul;
  int32_t last_rows;
};
hipError_t launch_fft_cols(const FftGrid& g, const ColTransform& ct, const double2* src, double2* a,
                           double2* b, double2** result, hipStream_t st);

// Inverse transform along x of rows 0 .. my - 1 of `in`, then map1[j][i] =
// fl32(Re(.) * scale) and (if map2) map2[j][i] = fl32(Im(.) * scale) for i < mx.
hipError_t launch_fft_rows_store(const FftGrid& g, const double2* in, int32_t mx, int32_t my,
                                 double scale, float* map1, float* map2, hipStream_t st);

}  // namespace morse
