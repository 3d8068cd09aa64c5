/*
 * morse.h -- C ABI of the MI355X (gfx950) map-build and trajectory-search library.
 *
 * Method: McDougall & Albrow (2015), "Microlensing Observations Rapid Search for
 * Exoplanets: MORSE code for GPUs".  The library builds a source-plane
 * magnification map of one binary lens by inverse ray shooting and searches source
 * trajectories over it, scoring each against a light curve.
 *
 * Conventions shared by every entry point
 *   - Units: angles on the sky in Einstein radii, times in days.
 *   - Lens placement (sec. 4.1): centre of mass at the origin, both masses on the x
 *     axis; separation s (the paper's d), mass ratio q = m2/m1 in [0, 1]; the primary
 *     m1 = 1/(1+q) sits at x1 = -s q/(1+q), the secondary at x2 = s/(1+q).
 *   - Pointers prefixed d_ are device memory on the context's device, h_ host memory.
 *     All buffers are owned by the caller; the library only reads h_ memory during
 *     the call.  The context owns a workspace it grows on demand.
 *   - Work is enqueued on the context's stream and is asynchronous unless stated.
 *   - Every entry point returns MORSE_OK (0) or a negative status; arguments are
 *     validated on the host before anything is enqueued, and a failing call
 *     enqueues nothing.  morse_last_error() gives a message.  Nothing aborts.
 *   - Not thread safe per context: use one context per host thread.
 */
#ifndef MORSE_H
#define MORSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MORSE_ABI_VERSION 7

enum morse_status {
  MORSE_OK = 0,
  MORSE_EINVAL = -1,       /* invalid argument (message says which) */
  MORSE_ENOMEM = -2,       /* device workspace allocation failed */
  MORSE_EHIP = -3,         /* a HIP runtime call failed */
  MORSE_ERANGE = -4,       /* a size limit would be exceeded (e.g. counts > 2^24) */
  MORSE_EUNSUPPORTED = -5  /* valid request that the library does not implement */
};

typedef struct morse_ctx morse_ctx;

/* A regular 2-D grid: centre (cx, cy), full widths (wx, wy), nx x ny cells, both
 * counts even and >= 2, widths finite and > 0.  Cell i spans
 * [cx - wx/2 + i wx/nx, cx - wx/2 + (i+1) wx/nx). */
typedef struct {
  double cx, cy, wx, wy;
  int32_t nx, ny;
} morse_grid2d;

int morse_abi_version(void);

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to enqueue on
 * (NULL: the context creates its own stream at default priority). */
int morse_ctx_create(int device, void* stream, morse_ctx** out);
/* Frees the workspace and the own stream (after synchronising it).  NULL is a no-op. */
int morse_ctx_destroy(morse_ctx* ctx);
/* Enqueue later work on `stream` (NULL: the device's null stream); waits for the
 * previous stream first when it changes. */
int morse_ctx_set_stream(morse_ctx* ctx, void* stream);
/* Blocks until all work enqueued on the context's stream has finished. */
int morse_ctx_synchronize(morse_ctx* ctx);
/* Message of the last failing call on ctx (ctx == NULL: on this host thread). */
const char* morse_last_error(const morse_ctx* ctx);

/* Kernel timing (a measurement aid, off by default).  Families of timed kernels: */
#define MORSE_KERNEL_RAYSHOOT 0 /* the ray-shooting kernel of morse_rayshoot / morse_build_map */
#define MORSE_KERNEL_SEARCH 1   /* the scoring kernel(s) of morse_search (batched: one launch) */
#define MORSE_KERNEL_GRADIENT 2 /* the chi-square/gradient kernel of morse_chi2_grad and of
                                   every round of morse_refine */
/* Enable timing for the families whose bit (1 << MORSE_KERNEL_*) is set in
 * kernel_mask (0 disables).  While a family is timed, each launch of its kernel is
 * bracketed by two HIP events recorded on the context's stream, and the entry points
 * that launch it enqueue their kernels one by one instead of replaying a captured
 * graph (same kernels, same results).  EINVAL for unknown bits. */
int morse_ctx_set_timing(morse_ctx* ctx, uint32_t kernel_mask);
/* Total event-measured time (ms) and number of timed launches of one family since the
 * last reset; waits for the pending events of every family.  reset != 0 zeroes the
 * family's totals after reading them.  Either output may be NULL. */
int morse_ctx_kernel_time(morse_ctx* ctx, int32_t kernel, double* h_total_ms,
                          int64_t* h_launches, int32_t reset);

/* ------------------------------------------------------------------------------
 * Map build (ray-shooting magnification maps, sec. 3; lens equation Eq. 2;
 * finite-source convolution, sec. 4.1).
 * --------------------------------------------------------------------------- */

/* Ray statistics of one build.  rays_in + rays_out + rays_nonfinite = rays_total;
 * rays_zero_axis counts binned rays that landed exactly on the window's horizontal
 * centre line (they break the exact mirror symmetry of the counts). */
typedef struct {
  uint64_t rays_total, rays_in, rays_out, rays_nonfinite, rays_zero_axis;
  uint32_t max_count;
  uint32_t reserved;
} morse_map_stats;

/* Inverse ray shooting (Eq. 2) of lattice rows [row_begin, row_end) of `rays` (the
 * image-plane lattice: ray (i, j) at cx + (i - nx/2 + 1/2) wx/nx, likewise y) into
 * the uint32 histogram d_counts[window.ny][window.nx] (row-major, y rows).
 * Arithmetic: binary32 without fused multiply-add and with correctly rounded
 * division, constants rounded once from FP64; bin rule symmetric about the window
 * centre (v = (zeta - c) nx/wx; v >= 0 -> nx/2 + floor(v), v < 0 ->
 * nx/2 - 1 - floor(-v), |v| >= nx/2 outside).  Counts are exact integers in any
 * launch order.  accumulate = 0 clears d_counts first.  d_stats (nullable, device
 * uint64[3]) accumulates {out of window, non-finite, on the centre line}.
 * Errors: EINVAL for bad grids, s <= 0, q outside [0, 1], bad row range. */
int morse_rayshoot(morse_ctx* ctx, double s, double q, const morse_grid2d* rays,
                   const morse_grid2d* window, int32_t row_begin, int32_t row_end,
                   uint32_t* d_counts, int32_t accumulate, uint64_t* d_stats);

/* Normalise counts to magnification and convolve with a uniform disk of radius rho
 * (sec. 4.1 convolution with a source profile).  A = scale * sum_k w_k c_{p+k}, with
 * scale = (hx hy)/(dx dy) (lattice cell over pixel area, hx the binary32 lattice
 * spacing) and w_k = area(disk(rho) ∩ pixel k)/(pi rho^2) renormalised to sum 1;
 * taps row-major over the stencil, neighbours beyond the edge clamp to the edge
 * pixel.  rho <= half a pixel reduces to A = c * scale.  Output float
 * d_map[window.ny][window.nx].  Errors: EINVAL (rho < 0 or not finite), ERANGE
 * (stencil wider than 31 pixels). */
int morse_normalize_convolve(morse_ctx* ctx, const uint32_t* d_counts, const morse_grid2d* rays,
                             const morse_grid2d* window, double rho, float* d_map);

/* build_map(s, q, window, rays): morse_rayshoot over all rows, then
 * morse_normalize_convolve.  d_counts may be NULL (workspace is used).  h_stats
 * (nullable) is filled after the context's stream is synchronised; max_count > 2^24
 * returns ERANGE (the FP32 normalisation would no longer be exact). */
int morse_build_map(morse_ctx* ctx, double s, double q, const morse_grid2d* rays,
                    const morse_grid2d* window, double rho, uint32_t* d_counts, float* d_map,
                    morse_map_stats* h_stats);

/* Finite-source maps for several source radii from one count map (sec. 4.1: each
 * point-source map is convolved with radially symmetric source profiles of several
 * radii and one fixed limb-darkening coefficient, giving one map per radius).
 * Profile: the linear limb-darkening law with unit mean brightness over the disk,
 * I(r) = 1 - gamma (1 - 1.5 sqrt(1 - r^2/rho^2)) for r <= rho; gamma = 0 is the
 * uniform disk.  Pixel weights w_k = (integral of I over pixel k ∩ disk)/(pi rho^2),
 * the area part from the circle-rectangle overlap and the limb part from closed-form
 * hemisphere volumes, renormalised to sum 1 in FP64.
 * For each k, d_maps + k * ny * nx receives A = scale * sum_k w_k c_{p+k} with the
 * scale and edge clamp of morse_normalize_convolve.  Two evaluations:
 *  - direct (stencil at most 31 x 31 and fewer than fft_min_taps non-zero taps): the
 *    binary32 sum of morse_normalize_convolve with binary32 weights, in the same tap
 *    order; for gamma = 0 identical bits to morse_normalize_convolve;
 *  - FFT otherwise: the counts, extended past the edges by their edge pixels, are
 *    convolved with the FP64 weights through FP64 transforms of power-of-two size
 *    (at least map + 2 R per side, at most 4096), the result rounded once to binary32
 *    (scale in FP64): within one binary32 unit in the last place of the FP64 direct
 *    sum, closer than the direct binary32 sum of a wide stencil.
 * fft_min_taps <= 0 takes MORSE_STACK_FFT_MIN_TAPS.  h_rho[n_rho] is host memory read
 * during the call.  The first call for a set of (radii, gamma, pixel size) computes
 * and keeps the profile transforms in the context (a synchronising call); later calls
 * enqueue kernels only.  Workspace: three transforms (16 B per padded pixel each) plus
 * one kept transform per pair of FFT radii.
 * Errors: EINVAL (gamma outside [0, 1], a radius negative or not finite, NULL
 * pointers), ERANGE (an FFT side above 4096). */
#define MORSE_STACK_FFT_MIN_TAPS 256
int morse_convolve_stack(morse_ctx* ctx, const uint32_t* d_counts, const morse_grid2d* rays,
                         const morse_grid2d* window, const double* h_rho, int32_t n_rho,
                         double gamma, int32_t fft_min_taps, float* d_maps);

/* The FP64 weights morse_convolve_stack uses for one radius (host only, no device
 * needed): stencil [2 ry + 1][2 rx + 1] (row = y offset) without all-zero outer
 * rings, normalised to sum 1.  Always sets *h_rx, *h_ry; writes h_w when it is not
 * NULL (capacity = its length in doubles).  Errors (message in morse_last_error(NULL)):
 * EINVAL (bad rho, pixel sizes or gamma; NULL h_rx / h_ry), ERANGE (capacity too
 * small, rho above 4096 pixels). */
int morse_profile_weights(double rho, double dx, double dy, double gamma, double* h_w,
                          int64_t capacity, int32_t* h_rx, int32_t* h_ry);

/* ------------------------------------------------------------------------------
 * Trajectory search (sec. 4.2: chi-square of each trajectory through a map by
 * bilinear interpolation; Eqs. 5-6: flux linear in magnification, so F_s and F_b are
 * profiled out by weighted least squares).
 * --------------------------------------------------------------------------- */

/* One map: device pointer to float[window.ny][window.nx] and its source-plane grid. */
typedef struct {
  const float* d_map;
  morse_grid2d window;
} morse_map_view;

/* Light curves of n_events events, concatenated (CSR).  Event e owns points
 * [h_offsets[e], h_offsets[e+1]), at least 3 and at most 2^28 each (longer events
 * return ERANGE: the kernels address an event's arrays with 32-bit byte offsets),
 * h_offsets[0] = 0, times non-decreasing.
 * d_t: binary32 offsets t - h_t_ref[e]; d_flux: FP64 flux; d_weight: FP64
 * w = 1/sigma^2 > 0.  h_offsets and h_t_ref are host arrays. */
typedef struct {
  int32_t n_events;
  int32_t reserved;
  const int64_t* h_offsets;
  const double* h_t_ref;
  const float* d_t;
  const double* d_flux;
  const double* d_weight;
} morse_lightcurves;

enum { MORSE_TRAJ_GRID = 0, MORSE_TRAJ_LIST = 1 };

/* Trajectories (t0, u0, tE, alpha): zeta(t) = tau (cos a, sin a) + u0 (-sin a, cos a),
 * tau = (t - t0)/tE, tE > 0.
 * GRID: product of host FP64 axes, shared by all events, trajectory index
 *   ((iu0 * n_alpha + ia) * n_t0 + it0) * n_tE + itE; t0 absolute.
 * LIST: n trajectories per event, device FP64 rows (t0, u0, tE, alpha); shared = 1:
 *   one list [n][4] for all events; shared = 0: [n_events][n][4]. */
typedef struct {
  int32_t kind;
  int32_t n_u0, n_alpha, n_t0, n_tE;
  int32_t shared;
  const double* h_u0;
  const double* h_alpha;
  const double* h_t0;
  const double* h_tE;
  int64_t n;
  const double* d_params;
} morse_trajectories;

/* Outputs, each nullable; n_traj = trajectories per event.
 *   d_chi2, d_fs, d_fb:      [n_events][n_maps][n_traj] chi2 and profiled F_s, F_b;
 *   d_best_chi2, d_best_idx: [n_events][n_maps] smallest (chi2, trajectory index);
 *   top_k > 0: d_topk_chi2, d_topk_idx [n_events][top_k], the top_k smallest
 *     (chi2, map * n_traj + traj) of each event in ascending order (NaN last).
 * chi2 = sum w (F - F_s A - F_b)^2 at the unconstrained minimiser (F_s, F_b); when
 * det = S_AA S_w - S_A^2 <= 1e-12 S_AA S_w, F_s = 0 and F_b = S_F/S_w. */
typedef struct {
  double* d_chi2;
  double* d_fs;
  double* d_fb;
  double* d_best_chi2;
  int64_t* d_best_idx;
  int32_t top_k;
  int32_t reserved;
  double* d_topk_chi2;
  int64_t* d_topk_idx;
} morse_search_out;

enum { MORSE_SEARCH_PLAIN = 0, MORSE_SEARCH_BATCHED = 1 };

/* search(map, lightcurve, traj_grid) over n_maps maps and all events.
 * PLAIN: one launch per (event, map).  BATCHED: one persistent launch over a work
 * queue of (event, map, trajectory block) items, captured once into a HIP graph
 * per argument set and replayed; tile shapes from the context's autotune table.  The
 * batched mode scores a trajectory list in an order grouped by direction (256 buckets
 * of alpha per list, a device counting sort each call; workspace 8 B per trajectory
 * and 1 KiB per list, lists of at most 16384 events), outputs staying in the list's
 * own order.  Both modes give bitwise identical results.  Errors: EINVAL (shapes, null
 * pointers, w <= 0 is not checked on device), EUNSUPPORTED (top_k > 4096). */
int morse_search(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                 const morse_lightcurves* lcs, const morse_trajectories* trajs, int32_t mode,
                 morse_search_out* out);

/* Autotune the batched search on this problem: times the candidate tile /
 * trajectory-block shapes, keeps the fastest in the context (used by later BATCHED
 * searches of the same shape class) and, if cache_path is not NULL, merges it into
 * that JSON file.  Synchronises.  h_best_config (nullable) receives the index. */
int morse_autotune(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                   const morse_lightcurves* lcs, const morse_trajectories* trajs,
                   const char* cache_path, int32_t* h_best_config);
/* Load the shape choices of an autotune cache file into the context (classes it
 * already holds are replaced).  Entries naming an unknown shape index are skipped.
 * h_loaded (nullable) receives the number of classes taken.  Errors: EINVAL (NULL
 * path), EUNSUPPORTED (file missing or unreadable).  Host only. */
int morse_autotune_load(morse_ctx* ctx, const char* cache_path, int32_t* h_loaded);

/* Candidates from a top-k result (sec. 4.4: the best grid solutions seed the next
 * stage): for every event e and rank r, the trajectory d_topk_idx[e][r] =
 * map * n_traj + traj of `trajs` is written as FP64 row d_params[e*top_k + r] =
 * (t0, u0, tE, alpha) with d_event = e and d_map_index = map.  Ranks with index -1
 * (events with fewer than top_k trajectories) get trajectory 0 of map 0.
 * Errors: EINVAL (shapes, NULL pointers). */
int morse_candidates_from_topk(morse_ctx* ctx, const morse_trajectories* trajs, int32_t n_events,
                               int32_t n_maps, int32_t top_k, const int64_t* d_topk_idx,
                               double* d_params, int32_t* d_event, int32_t* d_map_index);

/* ------------------------------------------------------------------------------
 * Caustic-centred trajectories (sec. 4.2: radial distances r from the centres of the
 * caustics, scaled by their sizes, and angles phi, in place of u0 about the lens
 * centre; Fig. 1) and the minimum-magnification filter (sec. 4.3, first optimisation:
 * a trajectory whose magnification along its path, read from the point-source map,
 * never reaches the minimum the light curve implies is discarded).
 * ------------------------------------------------------------------------------ */

/* The separate caustics of the binary lens (s, q) (host only, no device needed).
 * Critical points at nphi equally spaced phases (the quartic m1 (z - x2)^2 +
 * m2 (z - x1)^2 = e^{-i phi} (z - x1)^2 (z - x2)^2, roots by the Aberth-Ehrlich
 * iteration); each is joined to the nearest critical point of the next phase and each
 * connected set is one critical curve, mapped by Eq. 2 to one caustic.  Rows of
 * h_out[n][5]: (cx, cy, half_w, half_h, size) of the caustic's bounding box, size =
 * the larger half-side; ordered by (round(1e9 cy), cx).  *h_n = the number of
 * caustics (1, 2 or 3); h_out may be NULL to ask for it.  Errors (morse_last_error(NULL)):
 * EINVAL (s <= 0, q outside (0, 1], nphi outside [16, 2^20], h_n NULL), ERANGE
 * (capacity < n). */
int morse_caustics(double s, double q, int32_t nphi, double* h_out, int32_t capacity, int32_t* h_n);

/* Lines (host only): for caustic k (rows of morse_caustics), r_j and phi_l,
 * h_lines[(k n_r + j) n_phi + l] = (u0, alpha, shift) with alpha = phi,
 * u0 = r S - cx sin phi + cy cos phi, shift = cx cos phi + cy sin phi: the path
 * zeta = tau (cos a, sin a) + u0 (-sin a, cos a) passes at r S from the caustic centre,
 * closest at tau = shift.  Errors: EINVAL (negative counts, NULL arrays). */
int morse_caustic_lines(const double* h_caustics, int32_t n_caustics, const double* h_r, int32_t n_r,
                        const double* h_phi, int32_t n_phi, double* h_lines);

/* Minimum-magnification filter of n lines d_lines[n][3] (device FP64, as above) on one
 * point-source map.  Each line is sampled across the map window: tau_k = fl32(tau_c -
 * R) + k fl32(2R/(n_s - 1)) in binary32 for k < n_s = ceil(2 R kmax) + 1, with tau_c =
 * cx cos a + cy sin a (window centre), R half the window diagonal and kmax the larger
 * of nx/wx, ny/wy (samples at most a pixel apart); each sample is evaluated exactly as
 * morse_search evaluates a point (t0' = 0, 1/tE = 1).  d_best[n] (float) = the largest
 * sample (NaN if any is NaN), d_keep[n] (uint8) = d_best >= fl32(a_min).  Optional:
 * d_kept[n] (int64) receives the kept line indices in ascending order, d_count (device
 * int64) their number, h_count the same on the host (synchronises).  Workspace: the map
 * packed into cells (16 B per pixel).  Errors: EINVAL (bad window, NULL arrays, a_min
 * not finite), ERANGE (map too large to pack, more than 1e7 samples per line). */
int morse_line_filter(morse_ctx* ctx, const morse_map_view* map, const double* d_lines, int64_t n,
                      double a_min, float* d_best, uint8_t* d_keep, int64_t* d_kept,
                      int64_t* d_count, int64_t* h_count);

/* Peak library and peak-count rejection (sec. 4.3, third optimisation: a trajectory is
 * rejected when its point-source magnification has fewer than the required number of
 * peaks, a peak being where the magnification gradient changes from positive to
 * negative) on the samples of morse_line_filter.  Scanning the samples in order: the
 * first sample starts a trough m; a rise is a sample a > fl32(m fl32(1 + h)); after a
 * rise the running maximum M (the first of equal maxima) becomes a peak when a sample
 * a < fl32(M fl32(1 - h)) follows, which starts the next trough (h = hysteresis in
 * [0, 1), relative; h = 0 is the literal rule, h > 0 keeps the counting noise of a
 * ray-shooting map from making peaks).  Outputs, device: d_best [n] as the filter,
 * d_npeaks [n] (int32) the peak count, d_peak_tau / d_peak_A [n][max_peaks] (float) the
 * position tau along the line (from its t0 point: the M_p of Eqs. 7-8) and value of the
 * first max_peaks peaks (NaN past the count), d_keep [n] = d_best >= fl32(a_min) and
 * d_npeaks >= min_peaks (the first and third optimisations together); d_kept, d_count,
 * h_count as the filter.  Workspace as the filter.  Errors: as the filter, EINVAL
 * (hysteresis outside [0, 1), max_peaks outside [1, 64], min_peaks < 0). */
int morse_line_peaks(morse_ctx* ctx, const morse_map_view* map, const double* d_lines, int64_t n,
                     double a_min, int32_t min_peaks, double hysteresis, int32_t max_peaks,
                     float* d_best, int32_t* d_npeaks, float* d_peak_tau, float* d_peak_A,
                     uint8_t* d_keep, int64_t* d_kept, int64_t* d_count, int64_t* h_count);

/* Simplex starts from observed peak times (sec. 4.3, fourth and fifth optimisations):
 * for k < n, line l = d_kept[k] (k when d_kept is NULL) of the peak library above
 * (max_peaks per line), d_start[k] = (t0', tE) in FP64 with t0' = t0 + shift tE:
 * n_tp = 1 (h_tp[0] = t_p, tE given): the line's highest peak M_p (ties: the earlier),
 * t0 = t_p - M_p tE (Eq. 7); n_tp = 2 (h_tp[0] < h_tp[1]): its two highest peaks in tau
 * order M_1 < M_2, tE = (t_p2 - t_p1)/(M_2 - M_1) (Eq. 8), t0 = t_p1 - M_1 tE.  Lines
 * with fewer stored peaks than n_tp get (NaN, NaN).  Errors: EINVAL (n < 0, n_tp not 1
 * or 2, times not finite and increasing, tE <= 0 with n_tp = 1, NULL arrays). */
int morse_peak_starts(morse_ctx* ctx, const double* d_lines, const int64_t* d_kept, int64_t n,
                      const int32_t* d_npeaks, const float* d_peak_tau, const float* d_peak_A,
                      int32_t max_peaks, const double* h_tp, int32_t n_tp, double tE,
                      double* d_start);

/* Trajectory list of the kept lines: d_params[(k n_t0 + a) n_tE + b][4] =
 * (t0_a - shift tE_b, u0, tE_b, alpha) of line d_kept[k] (line k when d_kept is NULL),
 * k < n_kept: t0 is the time of closest approach to the caustic centre.  The result is
 * a morse_trajs list (kind MORSE_TRAJ_LIST).  h_t0, h_tE host arrays (read during the
 * call; the call synchronises).  Errors: EINVAL (negative counts, NULL arrays, tE <= 0). */
int morse_lines_to_trajectories(morse_ctx* ctx, const double* d_lines, const int64_t* d_kept,
                                int64_t n_kept, const double* h_t0, int32_t n_t0, const double* h_tE,
                                int32_t n_tE, double* d_params);

/* Downhill simplex along lines (sec. 4.2: each (r, phi) trajectory runs a simplex for
 * the chi-square minimum over its times; sec. 5: up to 5000 steps).  One simplex per
 * (line, map) over x = (t0', ln tE), t0' the time of closest approach to the caustic
 * centre (the trajectory is (t0' - shift tE, u0, tE, alpha) of line (u0, alpha,
 * shift)), from d_start[line] = (t0', tE) and the vertices x0 + (step_t0, 0),
 * x0 + (0, step_ln_tE).  Reflection 1, expansion 2, contraction 1/2, shrink 1/2 with
 * the acceptance rules of Lagarias et al. (1998); vertices in a stable chi-square order
 * (a new vertex after old ones of equal value, NaN as +inf); stop when f_worst -
 * f_best <= ftol |f_best| or after max_iter iterations.  Chi-square as morse_search
 * computes it, for light curve `event`.  Outputs [n_lines][n_maps]: the best vertex's
 * chi-square, t0', tE, the iterations taken and (d_evals, nullable) the chi-square
 * evaluations made (3 initial, then 1 to 4 per iteration).  d_lines [n_lines][3] and d_start
 * [n_lines][2] are device FP64.  Several maps (a finite-source stack) give the source
 * radius as a map index.  The lines start in descending order of their largest sample
 * on the first map (the line filter's maximum, bucketed by log2), since high peaks take
 * the most steps; results do not depend on the order.  Workspace: 8 B per line + 4 KiB
 * beyond the packed maps.  Errors: EINVAL (as morse_chi2_grad; bad event, opts, NULL
 * arrays), ERANGE (maps too large to pack). */
typedef struct {
  int32_t max_iter; /* 5000 */
  int32_t reserved;
  double step_t0, step_ln_tE, ftol;
} morse_simplex_opts;
int morse_line_simplex(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                       const morse_lightcurves* lcs, int32_t event, const double* d_lines,
                       int64_t n_lines, const double* d_start, const morse_simplex_opts* opts,
                       double* d_chi2, double* d_t0, double* d_tE, int32_t* d_iters,
                       int32_t* d_evals);

/* ------------------------------------------------------------------------------
 * Finite-source magnification without maps (sec. 5: image-centred ray shooting).
 * --------------------------------------------------------------------------- */

typedef struct {
  int32_t n_b;      /* source boundary points (192) */
  int32_t n_crit;   /* critical-curve phases (1024; 4 critical points each) */
  int32_t n_side;   /* samples per region side in the growth test (128) */
  int32_t n_grow;   /* growth rounds at most (40) */
  int32_t n_r;      /* radial segments per region (256) */
  int32_t n_theta;  /* angular columns per region (256) */
  int32_t n_shrink; /* cuts of a region to its inside cells (2) */
  int32_t reserved;
  double near;      /* point source beyond near * rho from the caustic (10) */
  double gap;       /* angle gap (rad) and relative radius gap that separate regions (0.2) */
} morse_fs_opts;

/* Finite-source magnification of n sources d_zeta[n][2] (device FP64 positions, lens
 * centre of mass at the origin, masses on the x axis as morse_build_map) of radius rho
 * with the limb-darkened profile I = 1 - gamma (1 - 1.5 sqrt(1 - r^2/rho^2)) (gamma = 0:
 * uniform), binary lens (s, q).  As in sec. 5: a source whose centre lies more than
 * near * rho from every caustic point (the Eq. 2 images of the critical points at
 * n_crit phases) takes the point-source magnification of its images (the quintic of
 * Eq. 2; Eqs. 3-4).  Otherwise the images of its centre and of n_b boundary points and
 * the critical points whose caustic image lies inside it are seeds, in polar
 * coordinates (r, theta) about the centre of mass; the seeds sorted by theta are cut at
 * gaps wider than gap, each run sorted by r is cut where consecutive radii differ by
 * more than max(gap r, 4 rho); each run is a region [r0, r1] x [t0, t1], padded by 10 %
 * of its extent plus rho (r) and rho / r1 (theta), grown (a side with any of n_side
 * samples mapping inside the source moves out by a quarter extent, at most n_grow
 * rounds; 2 pi in theta makes a ring); overlapping regions merge; each region is
 * integrated over n_theta columns of n_r radial segments (f = rho^2 - |zeta(z) -
 * zeta_s|^2 linear along a segment, the limb at f = 0, the square root of the profile
 * integrated exactly for linear f), cut to its inside cells one cell wider and
 * integrated again (n_shrink times); A = the integral over pi rho^2.  Outputs, device:
 * d_A [n] (FP64), d_nreg [n] (int32, nullable): -1 point source, >= 1 regions, -2 more
 * than 2048 seeds, -3 more than 64 regions (A is NaN for -2 and -3).  All arithmetic
 * FP64.  The critical points stay resident in the context (32 B each) until a call needs
 * another (s, q, n_crit); workspace 8 B per source plus 2.8 KiB per source for at most
 * 4096 of them (11 MiB).  The call synchronises the context's stream once (it reads
 * the number of sources near a caustic, which sizes the image-centred passes: at most
 * 4096 sources each), so it cannot be captured into a graph.  Errors: EINVAL (s, q, rho, gamma
 * outside their ranges, opts out of range, NULL arrays), ERANGE (n > 2^31). */
int morse_fs_magnification(morse_ctx* ctx, double s, double q, const double* d_zeta, int64_t n,
                           double rho, double gamma, const morse_fs_opts* opts, double* d_A,
                           int32_t* d_nreg);

/* Source positions of one trajectory at n times (sec. 4.1 parameters; the trajectory
 * form of morse_search): h_params = (t0, u0, tE, alpha) host FP64, d_t [n] device FP64
 * times, d_zeta [n][2] = tau (cos alpha, sin alpha) + u0 (-sin alpha, cos alpha) with
 * tau = (t - t0)/tE, FP64 (the input of morse_fs_magnification for a light curve).
 * Errors: EINVAL (non-finite parameters, tE <= 0, NULL arrays, n < 0). */
int morse_trajectory_positions(morse_ctx* ctx, const double* h_params, const double* d_t, int64_t n,
                               double* d_zeta);

/* ------------------------------------------------------------------------------
 * Gradient and refinement (candidates from the search refined on their maps).
 * --------------------------------------------------------------------------- */

/* chi2 and d chi2/d (t0, u0, tE, alpha) of n candidates: d_params [n][4] FP64
 * natural parameters, candidate i on map d_map_index[i] for event d_event[i].
 * Gradient by the envelope theorem (F_s, F_b are exact minimisers):
 * -2 F_s sum w r dA/dtheta, r = F - F_s A - F_b, through the bilinear sample (or the
 * single-lens magnification off the map).  Samples as in morse_search; sums FP64.
 * Outputs (device, nullable): d_chi2 [n], d_grad [n][4], d_fs [n], d_fb [n].
 * Candidates are evaluated grouped by (map, event) (a device counting sort; by map
 * alone past 2^20 pairs), so that the GPU samples one map at a time; the order changes
 * the schedule only, never a result.  Workspace: 48 B per candidate + 4 B per
 * (map, event) pair. */
int morse_chi2_grad(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                    const morse_lightcurves* lcs, int64_t n, const double* d_params,
                    const int32_t* d_event, const int32_t* d_map_index, double* d_chi2,
                    double* d_grad, double* d_fs, double* d_fb);

/* morse_chi2_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same arguments,
 * kernels and results, with no hipMalloc, hipFree or allocating library call; the
 * context must already exist.  Its scratch (event offsets, reference times and map
 * table, the light-curve preparation, candidate constants and the packed cells of every
 * map: 24 B per event + 8 B per point + 48 B per candidate + 4 B per (map, event)
 * pair + 16 B per map cell, each part rounded up to 256 B, plus the table) lives in one static device array of
 * 128 MiB on each GPU the library runs on, held until the process ends.  Every call on
 * a GPU shares that GPU's array and leaves its contents there, so calls that overlap on
 * one GPU (other streams or contexts) race; calls on one stream are ordered.  The host
 * metadata is copied into the array on every call (host-synchronous copies from the
 * caller's arrays).  Errors: as morse_chi2_grad, and ERANGE when the scratch would
 * exceed 128 MiB (e.g. more than one 2048^2 map with long light curves). */
int morse_chi2_grad_noalloc(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                            const morse_lightcurves* lcs, int64_t n, const double* d_params,
                            const int32_t* d_event, const int32_t* d_map_index, double* d_chi2,
                            double* d_grad, double* d_fs, double* d_fb);

typedef struct {
  int32_t steps;    /* evaluation rounds after the initial one (e.g. 50) */
  int32_t history;  /* L-BFGS memory m, 1..16 */
  int32_t max_ls;   /* failed Armijo trials before a candidate stops */
  int32_t reserved;
  double c1;        /* Armijo constant, in (0, 1) */
  double shrink;    /* step reduction per failed trial, in (0, 1) */
} morse_lbfgs_opts;

/* refine(...): batched L-BFGS on p (binary32), the scaled displacement from each
 * candidate's start (t0 = t0_i + p0 tE_i, u0 = u0_i + p1, tE = tE_i exp(p2),
 * alpha = alpha_i + p3), with FP64 chi2 and gradients from the adjoint above.  One
 * round = one evaluation of every active candidate, then one update: round 0 accepts
 * p = 0; later rounds accept the trial if f_t <= f + c1 t (g.d) (storing the pair
 * s = p_t - p, y = g_t - g when s.y > 1e-12 |s||y|), else halve-by-`shrink` the
 * step t, stopping the candidate after max_ls failures.  After an accept the new
 * direction is the two-loop recursion d = -H g with H0 = (s.y / y.y) I of the newest
 * pair, or -(1e-2/|g|) g with no pairs or no descent; t = 1, p_t = fl32(p + t d).
 * Dot products are left-to-right FP64 without fused multiply-add.  d_params
 * [n][4] FP64 is read as the start and overwritten with the refined parameters;
 * d_chi2_out [n] receives the final chi2, d_chi2_init [n] (nullable) the initial.
 * Candidates are independent: with 1024 or more, the two halves run as two chains of
 * launches, one on the context's stream and one on a second stream of the context that
 * starts after the work already enqueued and that the context's stream waits for at
 * the end (results identical to one chain).  Each chain evaluates its candidates
 * grouped by (map, event), as morse_chi2_grad. */
int morse_refine(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                 const morse_lightcurves* lcs, int64_t n, double* d_params,
                 const int32_t* d_event, const int32_t* d_map_index,
                 const morse_lbfgs_opts* opts, double* d_chi2_out, double* d_chi2_init);

#ifdef __cplusplus
}
#endif

#endif /* MORSE_H */
