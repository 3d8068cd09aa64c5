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
};

hipError_t launch_line_simplex(const SimplexArgs& a, hipStream_t st);

}  // namespace morse
