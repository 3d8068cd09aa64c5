// C ABI, candidates: chi-square and gradient, batched L-BFGS refinement, and the
// downhill simplex along lines, all on candidates' own maps and light curves.

#include "host.h"

#include <mutex>

using namespace morse;
using namespace morse::host;

// Scratch of the allocation-free entry point (morse_chi2_grad_noalloc): one array per
// GPU, held until the process ends.  Host code uses its device address from
// hipGetSymbolAddress (kept per device), never the array's name.
constexpr size_t kNoallocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

namespace morse {
namespace host {
// Called by morse_ctx_create with `device` current (and again, cached, by the entry
// point).
int noalloc_scratch(int device, char** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(nullptr, MORSE_EUNSUPPORTED, "device %d: at most %d devices", device,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, MORSE_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[device];
  return MORSE_OK;
}
}  // namespace host
}  // namespace morse

namespace {

int plan_candidates(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                    const morse_lightcurves* lcs, int64_t n, Plan& pl, size_t& i_sums,
                    size_t& i_wF, size_t& i_quad) {
  if (!maps || n_maps <= 0) return fail(ctx, MORSE_EINVAL, "need n_maps >= 1 maps");
  int rc;
  for (int i = 0; i < n_maps; ++i) {
    if (!maps[i].d_map) return fail(ctx, MORSE_EINVAL, "map %d: d_map is NULL", i);
    if ((rc = check_window(ctx, &maps[i].window, "map window"))) return rc;
  }
  if ((rc = check_lightcurves(ctx, lcs))) return rc;
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if ((rc = check_quad_size(ctx, maps, n_maps))) return rc;
  i_sums = pl.add(24 * (size_t)lcs->n_events);
  i_wF = pl.add(8 * (size_t)lcs->h_offsets[lcs->n_events]);
  i_quad = pl.add(quad_region_bytes(maps, n_maps));
  return MORSE_OK;
}

// Host metadata of the candidate entry points (event offsets, reference times, map
// table) lives in its own device buffer, uploaded only when it changes, so calls that
// alternate with searches neither re-upload nor wait for the device.
int setup_candidates(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                     const morse_lightcurves* lcs, const Plan& pl, size_t i_sums, size_t i_wF,
                     size_t i_quad, LcView& lc, MapC*& d_maps) {
  int rc;
  const int32_t ne = lcs->n_events;
  std::vector<MapC> hm(n_maps);
  for (int i = 0; i < n_maps; ++i) hm[i] = make_mapc(maps[i].d_map, maps[i].window);
  assign_quads(hm, pl.ptr(ctx, i_quad));
  const size_t b_off = (8 * (size_t)(ne + 1) + 255) & ~size_t(255);
  const size_t b_tref = (8 * (size_t)ne + 255) & ~size_t(255);
  if ((rc = reserve_meta(ctx, ctx->cmeta, b_off + b_tref + sizeof(MapC) * n_maps))) return rc;
  int64_t* d_off = (int64_t*)ctx->cmeta.p;
  double* d_tref = (double*)(ctx->cmeta.p + b_off);
  d_maps = (MapC*)(ctx->cmeta.p + b_off + b_tref);
  Hasher h;
  h.pod(ctx->cmeta.p);
  h.pod(ne);
  h.pod(n_maps);
  h.bytes(lcs->h_offsets, 8 * (size_t)(ne + 1));
  h.bytes(lcs->h_t_ref, 8 * (size_t)ne);
  h.bytes(hm.data(), sizeof(MapC) * n_maps);  // includes the packed-cell addresses
  if (h.h != ctx->cmeta.key) {
    ctx->cmeta.key = 0;
    if ((rc = upload(ctx, d_off, lcs->h_offsets, 8 * (size_t)(ne + 1)))) return rc;
    if ((rc = upload(ctx, d_tref, lcs->h_t_ref, 8 * (size_t)ne))) return rc;
    if ((rc = upload(ctx, d_maps, hm.data(), sizeof(MapC) * n_maps))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // host arrays go out of scope
    ctx->cmeta.key = h.h;
  }
  lc.t = lcs->d_t;
  lc.w = lcs->d_weight;
  lc.F = lcs->d_flux;
  lc.wFc = (double*)pl.ptr(ctx, i_wF);
  lc.off = d_off;
  lc.sums = (double*)pl.ptr(ctx, i_sums);
  lc.t_ref = d_tref;
  HIP_TRY(ctx, launch_quad_pack(d_maps, hm.data(), n_maps, ctx->stream));
  HIP_TRY(ctx, launch_lc_prep(lc.t, lc.F, lc.w, lc.off, ne, (double*)lc.wFc, (double*)lc.sums,
                              ctx->stream));
  return MORSE_OK;
}
}  // namespace

namespace {

// Refinements of at least kRefineSplitMin candidates run as two chains on two streams,
// others as one captured graph.
constexpr int64_t kRefineSplitMin = 1024;

// Views of the candidates [c0, c0 + n) of a refinement's state and evaluation arguments.
LbfgsState part_state(const LbfgsState& s, int64_t c0, int64_t n) {
  LbfgsState r = s;
  r.n = n;
  r.anchor = s.anchor + 4 * c0;
  r.p = s.p + 4 * c0;
  r.pt = s.pt + 4 * c0;
  r.f = s.f + c0;
  r.g = s.g + 4 * c0;
  r.d = s.d + 4 * c0;
  r.step = s.step + c0;
  r.S = s.S + 4 * (int64_t)s.m * c0;
  r.Y = s.Y + 4 * (int64_t)s.m * c0;
  r.R = s.R + (int64_t)s.m * c0;
  r.nhist = s.nhist + c0;
  r.nls = s.nls + c0;
  r.active = s.active + c0;
  return r;
}

GradArgs part_args(const GradArgs& a, int64_t c0, int64_t n) {
  GradArgs r = a;
  r.n = n;
  if (a.params) r.params = a.params + 4 * c0;
  if (a.anchor) r.anchor = a.anchor + 4 * c0;
  if (a.pt) r.pt = a.pt + 4 * c0;
  if (a.active) r.active = a.active + c0;
  r.event = a.event + c0;
  r.mapidx = a.mapidx + c0;
  r.tc = a.tc + c0;
  r.tEv = a.tEv + c0;
  if (a.chi2) r.chi2 = a.chi2 + c0;
  if (a.grad) r.grad = a.grad + 4 * c0;
  if (a.fs) r.fs = a.fs + c0;
  if (a.fb) r.fb = a.fb + c0;
  if (a.order) r.order = a.order + c0;  // each part's order holds its own local indices
  return r;
}

}  // namespace

extern "C" {


int morse_line_simplex(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                       const morse_lightcurves* lcs, int32_t event, const double* d_lines,
                       int64_t n_lines, const double* d_start, const morse_simplex_opts* opts,
                       double* d_chi2, double* d_t0, double* d_tE, int32_t* d_iters,
                       int32_t* d_evals) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  Plan pl;
  size_t i_sums, i_wF, i_quad;
  if ((rc = plan_candidates(ctx, maps, n_maps, lcs, n_lines, pl, i_sums, i_wF, i_quad))) return rc;
  if (event < 0 || event >= lcs->n_events) return fail(ctx, MORSE_EINVAL, "event %d out of range", event);
  if (!opts) return fail(ctx, MORSE_EINVAL, "opts is NULL");
  if (opts->max_iter < 0) return fail(ctx, MORSE_EINVAL, "max_iter < 0");
  if (!(std::isfinite(opts->step_t0) && std::isfinite(opts->step_ln_tE) && std::isfinite(opts->ftol) &&
        opts->ftol >= 0.0))
    return fail(ctx, MORSE_EINVAL, "steps and ftol must be finite, ftol >= 0");
  if (n_lines == 0) return MORSE_OK;
  if (!d_lines || !d_start || !d_chi2 || !d_t0 || !d_tE || !d_iters)
    return fail(ctx, MORSE_EINVAL, "NULL device array");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // start order: lines by descending largest sample on the first map (the filter's
  // sampling of the line across the window)
  const morse_grid2d& w0 = maps[0].window;
  const double R = 0.5 * std::sqrt(w0.wx * w0.wx + w0.wy * w0.wy);
  const double ns64 = std::ceil(2.0 * R * std::max(w0.nx / w0.wx, w0.ny / w0.wy)) + 1.0;
  const bool ordered = ns64 <= 1.0e7 && n_lines <= INT32_MAX;
  const size_t i_key = pl.add(ordered ? 4 * (size_t)n_lines : 0),
               i_hist = pl.add(ordered ? 4 * (size_t)kSimplexPrioBins : 0),
               i_order = pl.add(ordered ? 4 * (size_t)n_lines : 0);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  SimplexArgs a{};
  MapC* d_maps;
  if ((rc = setup_candidates(ctx, maps, n_maps, lcs, pl, i_sums, i_wF, i_quad, a.lc, d_maps))) return rc;
  a.maps = d_maps;
  a.n_maps = n_maps;
  a.event = event;
  a.n_points = (int32_t)(lcs->h_offsets[event + 1] - lcs->h_offsets[event]);
  a.lines = d_lines;
  a.n_lines = n_lines;
  a.start = d_start;
  a.d_t0 = opts->step_t0;
  a.d_ln_tE = opts->step_ln_tE;
  a.ftol = opts->ftol;
  a.max_iter = opts->max_iter;
  a.chi2 = d_chi2;
  a.t0 = d_t0;
  a.tE = d_tE;
  a.iters = d_iters;
  a.evals = d_evals;
  if (ordered) {
    HIP_TRY(ctx, launch_simplex_order(a, w0.cx, w0.cy, R, (int32_t)ns64, (float)(2.0 * R / (ns64 - 1.0)),
                                      (uint32_t*)pl.ptr(ctx, i_key), (uint32_t*)pl.ptr(ctx, i_hist),
                                      (int32_t*)pl.ptr(ctx, i_order), ctx->stream));
    a.order = (const int32_t*)pl.ptr(ctx, i_order);
  }
  HIP_TRY(ctx, launch_line_simplex(a, ctx->stream));
  return MORSE_OK;
}

int morse_chi2_grad(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                    const morse_lightcurves* lcs, int64_t n, const double* d_params,
                    const int32_t* d_event, const int32_t* d_map_index, double* d_chi2,
                    double* d_grad, double* d_fs, double* d_fb) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  Plan pl;
  size_t i_sums, i_wF, i_quad;
  if ((rc = plan_candidates(ctx, maps, n_maps, lcs, n, pl, i_sums, i_wF, i_quad))) return rc;
  if (n > 0 && (!d_params || !d_event || !d_map_index))
    return fail(ctx, MORSE_EINVAL, "d_params / d_event / d_map_index is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const size_t i_tc = pl.add(sizeof(TrajC) * (size_t)n), i_tE = pl.add(8 * (size_t)n),
               i_order = pl.add(4 * (size_t)n), i_key = pl.add(4 * (size_t)n),
               i_hist = pl.add(4 * (size_t)order_bins(n_maps, lcs->n_events));
  if ((rc = reserve(ctx, pl.total()))) return rc;
  GradArgs a{};
  a.tc = (TrajC*)pl.ptr(ctx, i_tc);
  a.tEv = (double*)pl.ptr(ctx, i_tE);
  a.order = (const int32_t*)pl.ptr(ctx, i_order);
  MapC* d_maps;
  if ((rc = setup_candidates(ctx, maps, n_maps, lcs, pl, i_sums, i_wF, i_quad, a.lc, d_maps))) return rc;
  a.n = n;
  a.params = d_params;
  a.event = d_event;
  a.mapidx = d_map_index;
  a.maps = d_maps;
  a.n_events = lcs->n_events;
  a.n_maps = n_maps;
  a.chi2 = d_chi2;
  a.grad = d_grad;
  a.fs = d_fs;
  a.fb = d_fb;
  HIP_TRY(ctx, launch_cand_order(a, (uint32_t*)pl.ptr(ctx, i_key), (uint32_t*)pl.ptr(ctx, i_hist),
                                 (int32_t*)a.order, ctx->stream));
  HIP_TRY(ctx, launch_cand_prep(a, ctx->stream));
  LaunchTimer tm{ctx, MORSE_KERNEL_GRADIENT};
  HIP_TRY(ctx, tm.begin(ctx->stream));
  HIP_TRY(ctx, launch_chi2_grad(a, ctx->stream));
  HIP_TRY(ctx, tm.end(ctx->stream));
  return MORSE_OK;
}

int morse_chi2_grad_noalloc(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                            const morse_lightcurves* lcs, int64_t n, const double* d_params,
                            const int32_t* d_event, const int32_t* d_map_index, double* d_chi2,
                            double* d_grad, double* d_fs, double* d_fb) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  Plan pl;
  size_t i_sums, i_wF, i_quad;
  if ((rc = plan_candidates(ctx, maps, n_maps, lcs, n, pl, i_sums, i_wF, i_quad))) return rc;
  if (n > 0 && (!d_params || !d_event || !d_map_index))
    return fail(ctx, MORSE_EINVAL, "d_params / d_event / d_map_index is NULL");
  const int32_t ne = lcs->n_events;
  const size_t b_off = (8 * (size_t)(ne + 1) + 255) & ~size_t(255);
  const size_t b_tref = (8 * (size_t)ne + 255) & ~size_t(255);
  const size_t i_meta = pl.add(b_off + b_tref + sizeof(MapC) * n_maps);
  const size_t i_tc = pl.add(sizeof(TrajC) * (size_t)n), i_tE = pl.add(8 * (size_t)n),
               i_order = pl.add(4 * (size_t)n), i_key = pl.add(4 * (size_t)n),
               i_hist = pl.add(4 * (size_t)order_bins(n_maps, ne));
  if (pl.total() > kNoallocScratchBytes)
    return fail(ctx, MORSE_ERANGE,
                "needs %.1f MiB of scratch; the allocation-free entry point holds %zu MiB "
                "(packed maps, light-curve preparation and candidate constants)",
                pl.total() / 1048576.0, kNoallocScratchBytes >> 20);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  char* base = nullptr;
  if ((rc = noalloc_scratch(ctx->device, &base))) return fail(ctx, rc, "%s", morse_last_error(nullptr));
  // metadata: event offsets | reference times | map table, uploaded on every call (the
  // array keeps whatever the last call on this GPU left in it)
  std::vector<MapC> hm(n_maps);
  for (int i = 0; i < n_maps; ++i) hm[i] = make_mapc(maps[i].d_map, maps[i].window);
  assign_quads(hm, pl.ptr_at(base, i_quad));
  char* meta = pl.ptr_at(base, i_meta);
  MapC* d_maps = (MapC*)(meta + b_off + b_tref);
  if ((rc = upload(ctx, meta, lcs->h_offsets, 8 * (size_t)(ne + 1)))) return rc;
  if ((rc = upload(ctx, meta + b_off, lcs->h_t_ref, 8 * (size_t)ne))) return rc;
  if ((rc = upload(ctx, d_maps, hm.data(), sizeof(MapC) * n_maps))) return rc;
  GradArgs a{};
  a.lc.t = lcs->d_t;
  a.lc.w = lcs->d_weight;
  a.lc.F = lcs->d_flux;
  a.lc.wFc = (double*)pl.ptr_at(base, i_wF);
  a.lc.off = (const int64_t*)meta;
  a.lc.sums = (double*)pl.ptr_at(base, i_sums);
  a.lc.t_ref = (const double*)(meta + b_off);
  HIP_TRY(ctx, launch_quad_pack(d_maps, hm.data(), n_maps, ctx->stream));
  HIP_TRY(ctx, launch_lc_prep(a.lc.t, a.lc.F, a.lc.w, a.lc.off, ne, (double*)a.lc.wFc,
                              (double*)a.lc.sums, ctx->stream));
  a.tc = (TrajC*)pl.ptr_at(base, i_tc);
  a.tEv = (double*)pl.ptr_at(base, i_tE);
  a.order = (const int32_t*)pl.ptr_at(base, i_order);
  a.n = n;
  a.params = d_params;
  a.event = d_event;
  a.mapidx = d_map_index;
  a.maps = d_maps;
  a.n_events = ne;
  a.n_maps = n_maps;
  a.chi2 = d_chi2;
  a.grad = d_grad;
  a.fs = d_fs;
  a.fb = d_fb;
  HIP_TRY(ctx, launch_cand_order(a, (uint32_t*)pl.ptr_at(base, i_key), (uint32_t*)pl.ptr_at(base, i_hist),
                                 (int32_t*)a.order, ctx->stream));
  HIP_TRY(ctx, launch_cand_prep(a, ctx->stream));
  HIP_TRY(ctx, launch_chi2_grad(a, ctx->stream));
  return MORSE_OK;
}

int morse_refine(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                 const morse_lightcurves* lcs, int64_t n, double* d_params,
                 const int32_t* d_event, const int32_t* d_map_index,
                 const morse_lbfgs_opts* opts, double* d_chi2_out, double* d_chi2_init) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (!opts) return fail(ctx, MORSE_EINVAL, "opts is NULL");
  if (opts->steps < 0 || opts->steps > 100000 || opts->history < 1 || opts->history > 16 ||
      opts->max_ls < 1 || !(opts->c1 > 0 && opts->c1 < 1) || !(opts->shrink > 0 && opts->shrink < 1))
    return fail(ctx, MORSE_EINVAL, "invalid L-BFGS options");
  int rc;
  Plan pl;
  size_t i_sums, i_wF, i_quad;
  if ((rc = plan_candidates(ctx, maps, n_maps, lcs, n, pl, i_sums, i_wF, i_quad))) return rc;
  if (n > 0 && (!d_params || !d_event || !d_map_index || !d_chi2_out))
    return fail(ctx, MORSE_EINVAL, "d_params / d_event / d_map_index / d_chi2_out is NULL");
  if (n == 0) return MORSE_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int m = opts->history;
  const size_t i_anchor = pl.add(32 * n), i_p = pl.add(16 * n), i_pt = pl.add(16 * n),
               i_f = pl.add(8 * n), i_g = pl.add(32 * n), i_d = pl.add(32 * n), i_step = pl.add(8 * n),
               i_S = pl.add(32 * (size_t)n * m), i_Y = pl.add(32 * (size_t)n * m),
               i_R = pl.add(8 * (size_t)n * m), i_int = pl.add(12 * n), i_ft = pl.add(8 * n),
               i_gt = pl.add(32 * n), i_tc = pl.add(sizeof(TrajC) * (size_t)n),
               i_tE = pl.add(8 * (size_t)n), i_order = pl.add(4 * (size_t)n),
               i_key = pl.add(4 * (size_t)n);
  const int64_t nbins = order_bins(n_maps, lcs->n_events);
  const size_t i_hist0 = pl.add(4 * (size_t)nbins), i_hist1 = pl.add(4 * (size_t)nbins);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  GradArgs a{};
  a.tc = (TrajC*)pl.ptr(ctx, i_tc);
  a.tEv = (double*)pl.ptr(ctx, i_tE);
  MapC* d_maps;
  if ((rc = setup_candidates(ctx, maps, n_maps, lcs, pl, i_sums, i_wF, i_quad, a.lc, d_maps))) return rc;
  LbfgsState s;
  s.n = n;
  s.m = m;
  s.max_ls = opts->max_ls;
  s.c1 = opts->c1;
  s.shrink = opts->shrink;
  double* anchor = (double*)pl.ptr(ctx, i_anchor);
  s.anchor = anchor;
  s.p = (float*)pl.ptr(ctx, i_p);
  s.pt = (float*)pl.ptr(ctx, i_pt);
  s.f = (double*)pl.ptr(ctx, i_f);
  s.g = (double*)pl.ptr(ctx, i_g);
  s.d = (double*)pl.ptr(ctx, i_d);
  s.step = (double*)pl.ptr(ctx, i_step);
  s.S = (double*)pl.ptr(ctx, i_S);
  s.Y = (double*)pl.ptr(ctx, i_Y);
  s.R = (double*)pl.ptr(ctx, i_R);
  int32_t* ints = (int32_t*)pl.ptr(ctx, i_int);
  s.nhist = ints;
  s.nls = ints + n;
  s.active = ints + 2 * n;
  a.n = n;
  a.anchor = anchor;
  a.pt = s.pt;
  a.active = s.active;
  a.event = d_event;
  a.mapidx = d_map_index;
  a.maps = d_maps;
  a.n_events = lcs->n_events;
  a.n_maps = n_maps;
  double* ft = (double*)pl.ptr(ctx, i_ft);
  double* gt = (double*)pl.ptr(ctx, i_gt);
  a.chi2 = ft;
  a.grad = gt;
  a.order = (const int32_t*)pl.ptr(ctx, i_order);
  uint32_t* hist[2] = {(uint32_t*)pl.ptr(ctx, i_hist0), (uint32_t*)pl.ptr(ctx, i_hist1)};
  // The rounds are captured once per argument set and replayed: start (evaluation
  // order grouped by map, anchor copy, state reset, first-trial constants), steps + 1
  // rounds of (evaluation, update with the next trial's constants), write-back.
  Hasher h;
  h.pod(ctx->ws_epoch);
  h.pod(n);
  h.pod(n_maps);
  h.pod(lcs->n_events);
  h.pod(*opts);
  h.pod(d_params);
  h.pod(d_event);
  h.pod(d_map_index);
  h.pod(d_chi2_out);
  h.pod(d_chi2_init);
  h.pod(lcs->d_t);
  h.pod(lcs->d_flux);
  h.pod(lcs->d_weight);
  // everything the workspace layout and the metadata buffer depend on
  h.bytes(lcs->h_offsets, 8 * (size_t)(lcs->n_events + 1));
  for (int i = 0; i < n_maps; ++i) {
    h.pod(maps[i].d_map);
    h.pod(maps[i].window);
  }
  h.pod(ctx->cmeta.p);
  // start, steps + 1 rounds, write-back of the candidate ranges [c0[k], c0[k] + nc[k])
  // on streams cs[k], k < parts, their launches interleaved round by round; with
  // `timing`, events bracket each evaluation
  auto enqueue = [&](int parts, const hipStream_t* cs, const int64_t* c0, const int64_t* nc,
                     bool timing) -> hipError_t {
    LbfgsState sp[2];
    GradArgs ap[2];
    for (int k = 0; k < parts; ++k) {
      sp[k] = part_state(s, c0[k], nc[k]);
      ap[k] = part_args(a, c0[k], nc[k]);
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < parts && e == hipSuccess; ++k) {
      e = launch_cand_order(ap[k], (uint32_t*)pl.ptr(ctx, i_key) + c0[k], hist[k],
                            const_cast<int32_t*>(ap[k].order), cs[k]);
      if (e == hipSuccess)
        e = launch_refine_init(sp[k], ap[k], d_params + 4 * c0[k], anchor + 4 * c0[k], cs[k]);
    }
    for (int r = 0; r <= opts->steps && e == hipSuccess; ++r) {
      for (int k = 0; k < parts && e == hipSuccess; ++k) {
        LaunchTimer tm{ctx, MORSE_KERNEL_GRADIENT};
        if (timing) e = tm.begin(cs[k]);
        if (e == hipSuccess) e = launch_chi2_grad(ap[k], cs[k]);
        if (e == hipSuccess && timing) e = tm.end(cs[k]);
        double* init = (r == 0 && d_chi2_init) ? d_chi2_init + c0[k] : nullptr;
        if (e == hipSuccess)
          e = launch_lbfgs_update(sp[k], ap[k], r, ft + c0[k], gt + 4 * c0[k], init, cs[k]);
      }
    }
    for (int k = 0; k < parts && e == hipSuccess; ++k)
      e = launch_lbfgs_finish(sp[k], d_params + 4 * c0[k], d_chi2_out + c0[k], cs[k]);
    return e;
  };
  const int64_t whole0 = 0;
  if (timed(ctx, MORSE_KERNEL_GRADIENT)) {  // same kernels, launched one by one
    HIP_TRY(ctx, enqueue(1, &ctx->stream, &whole0, &n, true));
    return MORSE_OK;
  }
  if (n >= kRefineSplitMin) {
    // Candidates are independent: the two halves run as two chains of launches on two
    // streams, so that one chain's evaluations keep the GPU busy while the other waits
    // between its dependent launches.  Both chains start after the work already on the
    // context's stream, and the stream waits for both; once forked, the join is
    // recorded even if a launch failed, so later work never overlaps the second chain.
    const hipStream_t cs[2] = {ctx->stream, ctx->fork_stream};
    const int64_t c0[2] = {0, n / 2}, nc[2] = {n / 2, n - n / 2};
    HIP_TRY(ctx, hipEventRecord(ctx->fork_ev, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->fork_stream, ctx->fork_ev, 0));
    const hipError_t e = enqueue(2, cs, c0, nc, false);
    hipError_t ej = hipEventRecord(ctx->join_ev, ctx->fork_stream);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(ctx->stream, ctx->join_ev, 0);
    HIP_TRY(ctx, e);
    HIP_TRY(ctx, ej);
    return MORSE_OK;
  }
  if (!ctx->refine_gexec || ctx->refine_key != h.h) {
    if (ctx->refine_gexec) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      (void)hipGraphExecDestroy(ctx->refine_gexec);
      ctx->refine_gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    hipStream_t cs = ctx->capture_stream;
    HIP_TRY(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(1, &cs, &whole0, &n, false);
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(ctx, MORSE_EHIP, "refine graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&ctx->refine_gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ctx->refine_gexec = nullptr;
      return fail(ctx, MORSE_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    ctx->refine_key = h.h;
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->refine_gexec, ctx->stream));
  return MORSE_OK;
}

}  // extern "C"
