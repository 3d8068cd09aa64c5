// Launchers of the caustic-centred line kernels (lines.hip) used by api_lines.hip.  Not part
// of the public ABI.
#pragma once

#include "internal.h"

namespace morse {

struct LineFilterArgs {
  MapC m;                // the map, packed into cells
  const double* lines;   // [n][3] (u0, alpha, shift), FP64
  int64_t n;
  double cxw, cyw;       // window centre
  double half_diag;      // half the window diagonal
  int32_t ns;            // samples per line
  float h;               // binary32 sample spacing along the line
  float amin;            // binary32 threshold
  float* best;           // [n] largest sample per line
  uint8_t* keep;         // [n] best >= amin
};

hipError_t launch_line_filter(const LineFilterArgs& a, hipStream_t st);

// The filter's samples, their largest value and the peak library of each line: peaks
// with relative hysteresis (rise above fl32(trough * up), fall below fl32(top * down)),
// their count and the tau and value of the first kmax; keep = best >= amin and
// count >= min_peaks.
struct LinePeakArgs {
  LineFilterArgs f;
  float up, down;     // fl32(1 + h), fl32(1 - h)
  int32_t min_peaks;
  int32_t kmax;       // peaks stored per line
  int32_t* npeaks;    // [n]
  float* ptau;        // [n][kmax], NaN past the count
  float* pA;          // [n][kmax]
};
hipError_t launch_line_peaks(const LinePeakArgs& a, hipStream_t st);

// Simplex starts (t0', tE) of lines kept[k] (k when kept is null), k < n, from n_tp
// observed peak times (Eq. 7 with the highest peak and tE; Eq. 8 with the two highest).
struct PeakStartArgs {
  const double* lines;
  const int64_t* kept;
  int64_t n;
  const int32_t* npeaks;
  const float* ptau;
  const float* pA;
  int32_t kmax;
  int32_t n_tp;
  double tp1, tp2, tE;
  double* start;      // [n][2]
};
hipError_t launch_peak_starts(const PeakStartArgs& a, hipStream_t st);

// Indices of the set flags of keep[n], ascending, into kept[]; their number into
// *d_count.  scratch: compact_scratch_elems(n) int64 values.
size_t compact_scratch_elems(int64_t n);
hipError_t launch_compact(const uint8_t* keep, int64_t n, int64_t* scratch, int64_t* kept,
                          int64_t* d_count, hipStream_t st);

// params[(k n_t0 + a) n_tE + b] = (t0[a] - shift tE[b], u0, tE[b], alpha) of line
// kept[k] (line k when kept is null), k < n_kept.
hipError_t launch_lines_to_traj(const double* lines, const int64_t* kept, int64_t n_kept,
                                const double* t0, int32_t n_t0, const double* tE, int32_t n_tE,
                                double* params, hipStream_t st);

}  // namespace morse
