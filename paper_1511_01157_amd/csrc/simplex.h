// Launcher of the line-simplex kernel (simplex.hip) used by api_refine.hip.  Not part of the
// public ABI.
#pragma once

#include "internal.h"

namespace morse {

struct SimplexArgs {
  const MapC* maps;      // device [n_maps], packed cells
  int32_t n_maps;
  LcView lc;             // prepared light curves (wFc and per-event sums)
  int32_t event;         // the event every line is fitted to
  int32_t n_points;      // its number of points (host copy)
  const double* lines;   // [n_lines][3] (u0, alpha, shift)
  int64_t n_lines;
  const double* start;   // [n_lines][2] (t0', tE)
  double d_t0, d_ln_tE;  // initial simplex steps
  double ftol;
  int32_t max_iter;
  double* chi2;          // [n_lines][n_maps] outputs
  double* t0;
  double* tE;
  int32_t* iters;
  int32_t* evals;        // nullable: chi-square evaluations per item
  const int32_t* order;  // nullable: the lines in the order their workgroups start
};

hipError_t launch_line_simplex(const SimplexArgs& a, hipStream_t st);

// Start order of the simplex: lines by descending largest sample on the first map (the
// line filter's maximum, over ns samples h apart from the window centre's projection
// minus half_diag), bucketed by log2 into kSimplexPrioBins; lines with high peaks take
// the most steps, so starting them first shortens the launch.  Results do not depend
// on it.  key, hist, order: workspace of n_lines, kSimplexPrioBins and n_lines words.
constexpr int kSimplexPrioBins = 1024;
hipError_t launch_simplex_order(const SimplexArgs& a, double cxw, double cyw, double half_diag,
                                int32_t ns, float h, uint32_t* key, uint32_t* hist, int32_t* order,
                                hipStream_t st);

}  // namespace morse
