// Launchers of the image-centred finite-source magnification kernels (fsmag.hip) used by
// api_fsmag.hip.  Not part of the public ABI.
#pragma once

#include "internal.h"

namespace morse {

constexpr int kFsRegionCap = 64;  // regions per source
constexpr int kFsBatch = 4096;     // near sources per pass of the image-centred kernels

struct FsArgs {
  double m1, m2, x1, x2;     // lens (sec. 4.1 placement)
  const double* zeta;        // [n][2] source centres
  int64_t n;
  double rho, gamma;
  const double* crit;        // [n_crit][2] critical points
  const double* caus;        // [n_crit][2] their caustic images
  int32_t n_crit;
  int32_t n_b, n_side, n_grow, n_r, n_theta, n_shrink;
  double near, gap;
  double* A;                 // [n]
  int32_t* nreg;             // [n]: -1 point source, >= 1 regions, -2 seed capacity exceeded
  int32_t* near_list;        // [n] indices of the sources near a caustic (workspace)
  uint32_t* near_count;      // one counter (workspace, cleared by the launcher)
  // one batch of listed sources, near_list[item0 .. item0 + n_items) (workspace)
  int64_t item0, n_items;
  double* regs;              // [kFsBatch][kFsRegionCap][4] r0, r1, t0, t1
  int32_t* reg_count;        // [kFsBatch] regions per source, 0 after a failure
  double* reg_val;           // [kFsBatch][kFsRegionCap] each region's integral
  uint32_t* work;            // [kFsBatch * kFsRegionCap] (item, region) slots to integrate
  uint32_t* work_count;      // one counter (cleared by the launcher)
};

// zeta[i] = tau (cos alpha, sin alpha) + u0 (-sin alpha, cos alpha), tau = (t[i] - t0)/tE.
hipError_t launch_traj_positions(const double* t, int64_t n, double t0, double u0, double tE,
                                 double alpha, double* zeta, hipStream_t st);

// Caustic distance (one wavefront per source), then the point-source magnification of
// the far sources (one thread each); the sources within near * rho of the caustic are
// listed for the image-centred kernel.
hipError_t launch_fs_classify(const FsArgs& a, hipStream_t st);
// Image-centred magnification of the batch of listed sources: their regions (one
// workgroup per source), the region integrals with their shrink passes (one workgroup
// per region), then the sums per source.
hipError_t launch_fs_images(const FsArgs& a, int32_t max_blocks, hipStream_t st);

}  // namespace morse
