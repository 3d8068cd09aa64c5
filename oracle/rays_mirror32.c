/*
 * Inverse ray shooting into a source-plane histogram, FP32 mirror (plain C).
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Built with gcc
 * -O2 -ffp-contract=off (no fused multiply-add, SSE2 scalar FP32, round to nearest
 * even) so that every operation below is one correctly rounded IEEE binary32 op.
 *
 * What is computed (ray-shooting magnification maps, sec. 3 of McDougall & Albrow
 * 2015, using the binary-lens equation Eq. 2 with the lens placement of sec. 4.1):
 * every ray of a regular image-plane lattice is mapped to the source plane and
 * counted into the source-plane pixel it lands in.  The FP32 operation order and the
 * bin rule are the ones stated for the mirror in the oracle's Python module
 * oracle/rays.py (an independent numpy implementation of the same steps).
 *
 * Constants (computed by the caller in FP64 and rounded once to binary32):
 *   m1, m2, x1, x2  lens masses and positions;
 *   cx, cy, hx, hy  ray-lattice centre and spacing (h = W/N);
 *   sx, sy, kx, ky  window centre and pixels per Einstein radius (k = M/V).
 * Ray (i, j): x = cx + (i - Nx/2 + 1/2) hx, y likewise.
 *   d1 = x - x1, d2 = x - x2, yy = y*y, r1 = d1*d1 + yy, r2 = d2*d2 + yy,
 *   a1 = m1 / r1, a2 = m2 / r2,
 *   zx = (x - a1*d1) - a2*d2,  zy = (y - a1*y) - a2*y.
 * Bin: v = (z - s) * k; v >= 0 -> M/2 + floor(v) if v < M/2; v < 0 ->
 *   M/2 - 1 - floor(-v) if -v < M/2; otherwise outside.  Non-finite v -> nonfinite.
 * stats[0] rays out of window, stats[1] non-finite, stats[2] in-window rays with
 * v_y == 0 (they break the exact mirror symmetry of the histogram).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
  float m1, m2, x1, x2, cx, cy, hx, hy, sx, sy, kx, ky;
  int32_t nx, ny, mx, my;
} oracle_ray_params;

static int bin1(float v, int32_t m, int32_t* out) {
  float half = (float)(m / 2);
  if (v >= 0.0f) {
    if (v < half) { *out = m / 2 + (int32_t)floorf(v); return 1; }
    return 0;
  }
  float w = -v;
  if (w < half) { *out = m / 2 - 1 - (int32_t)floorf(w); return 1; }
  return 0;
}

typedef struct {
  const oracle_ray_params* p;
  int32_t j0, j1;
  uint32_t* counts;
  uint64_t stats[3];
} job_t;

static void* run_rows(void* arg) {
  job_t* job = (job_t*)arg;
  const oracle_ray_params* p = job->p;
  for (int32_t j = job->j0; j < job->j1; ++j) {
    float gy = (float)(j - p->ny / 2) + 0.5f;
    float y = p->cy + gy * p->hy;
    float yy = y * y;
    for (int32_t i = 0; i < p->nx; ++i) {
      float gx = (float)(i - p->nx / 2) + 0.5f;
      float x = p->cx + gx * p->hx;
      float d1 = x - p->x1;
      float d2 = x - p->x2;
      float r1 = d1 * d1 + yy;
      float r2 = d2 * d2 + yy;
      float a1 = p->m1 / r1;
      float a2 = p->m2 / r2;
      float t1 = a1 * d1;
      float t2 = a2 * d2;
      float zx = (x - t1) - t2;
      float u1 = a1 * y;
      float u2 = a2 * y;
      float zy = (y - u1) - u2;
      float vx = (zx - p->sx) * p->kx;
      float vy = (zy - p->sy) * p->ky;
      if (!isfinite(vx) || !isfinite(vy)) { job->stats[1]++; continue; }
      int32_t bx, by;
      if (!bin1(vx, p->mx, &bx) || !bin1(vy, p->my, &by)) { job->stats[0]++; continue; }
      if (vy == 0.0f) job->stats[2]++;
      job->counts[(size_t)by * (size_t)p->mx + (size_t)bx] += 1u;
    }
  }
  return NULL;
}

/* counts: caller-owned [my][mx] uint32, accumulated into (not cleared).
 * stats: uint64[3] accumulated into.  nthreads >= 1; rows are split evenly and each
 * thread uses a private histogram that is summed into counts at the end.
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_rayshoot_mirror32(const oracle_ray_params* p, uint32_t* counts, uint64_t* stats,
                             int32_t row_begin, int32_t row_end, int32_t nthreads) {
  if (!p || !counts || !stats || p->nx <= 0 || p->ny <= 0 || p->mx <= 0 || p->my <= 0 ||
      (p->nx & 1) || (p->ny & 1) || (p->mx & 1) || (p->my & 1) || row_begin < 0 ||
      row_end > p->ny || row_begin > row_end || nthreads < 1)
    return -1;
  size_t npx = (size_t)p->mx * (size_t)p->my;
  job_t* jobs = (job_t*)calloc((size_t)nthreads, sizeof(job_t));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -2; }
  int32_t rows = row_end - row_begin;
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].p = p;
    jobs[t].j0 = row_begin + (int32_t)((int64_t)rows * t / nthreads);
    jobs[t].j1 = row_begin + (int32_t)((int64_t)rows * (t + 1) / nthreads);
    jobs[t].counts = (t == 0) ? counts : (uint32_t*)calloc(npx, sizeof(uint32_t));
    if (!jobs[t].counts) {
      for (int u = 1; u < t; ++u) free(jobs[u].counts);
      free(jobs); free(th);
      return -2;
    }
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, run_rows, &jobs[t]);
  run_rows(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  for (int t = 0; t < nthreads; ++t) {
    for (int k = 0; k < 3; ++k) stats[k] += jobs[t].stats[k];
    if (t > 0) {
      for (size_t k = 0; k < npx; ++k) counts[k] += jobs[t].counts[k];
      free(jobs[t].counts);
    }
  }
  free(jobs);
  free(th);
  return 0;
}
