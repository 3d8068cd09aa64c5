// C ABI, trajectory search: plain and batched (persistent, graph-captured) searches,
// best-per-map and top-k selection, the autotuner of the batched shape and its cache,
// and candidate lists from the top-k.

#include "host.h"

using namespace morse;
using namespace morse::host;

namespace {

struct TuneCfg {
  int traj_per_item;
  int waves_per_block;
  int blocks_per_cu;
  int tu;
};
// Candidate shapes of the batched search tried by the autotuner; index 0 is the
// default before tuning.  traj_per_item = trajectories per wavefront work item,
// tu = trajectories scored together by one wavefront (sharing light-curve loads).
// The last two take one TU group per item (traj_per_item = tu), the fastest shapes on
// batches of many events and maps.
constexpr TuneCfg kTune[] = {
    {8, 4, 16, 2},  {8, 4, 16, 1},  {16, 4, 16, 2}, {8, 8, 8, 2},
    {32, 8, 8, 2},  {4, 4, 16, 2},  {16, 8, 4, 4},  {8, 2, 32, 2},
    {16, 4, 16, 4}, {32, 8, 8, 1},  {8, 2, 32, 1},  {64, 4, 8, 4},
    {32, 8, 4, 4},  {16, 4, 8, 4},  {8, 8, 4, 4},   {16, 8, 2, 4},
    {4, 8, 4, 4},   {4, 4, 8, 4},
};
constexpr int kNumTune = sizeof(kTune) / sizeof(kTune[0]);
// k_search_batched is compiled for at most 512 lanes (8 wavefronts) per workgroup and
// instantiated for TU = 1, 2 and 4; a shape outside that would not launch.
constexpr bool tune_shapes_valid() {
  for (const TuneCfg& c : kTune)
    if (c.waves_per_block < 1 || c.waves_per_block > 8 || c.blocks_per_cu < 1 ||
        c.traj_per_item < 1 || !(c.tu == 1 || c.tu == 2 || c.tu == 4))
      return false;
  return true;
}
static_assert(tune_shapes_valid(), "a batched-search shape the kernel cannot launch");


}  // namespace

// =============================================================================
// Search planning shared by search / autotune.
namespace {

struct SearchPlan {
  int64_t n_traj = 0;
  int32_t n_events = 0, n_maps = 0;
  int64_t n_pts = 0;
  TrajC* tc = nullptr;
  MapC* d_maps = nullptr;
  std::vector<MapC> h_maps;
  LcView lc{};
  double* chi2 = nullptr;  // output or workspace
  void* tk_scratch = nullptr;
  int num_cu = 256;
  uint32_t* counter = nullptr;
  double* axes = nullptr;
  // trajectory lists: scoring order of the batched kernel and its counting-sort counters
  int32_t* perm = nullptr;
  uint32_t* perm_key = nullptr;
  uint32_t* perm_hist = nullptr;
  int32_t perm_lists = 0;
};

int validate_search(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                    const morse_lightcurves* lcs, const morse_trajectories* trajs) {
  int rc;
  if (!maps || n_maps <= 0) return fail(ctx, MORSE_EINVAL, "need n_maps >= 1 maps");
  for (int i = 0; i < n_maps; ++i) {
    if (!maps[i].d_map) return fail(ctx, MORSE_EINVAL, "map %d: d_map is NULL", i);
    if ((rc = check_window(ctx, &maps[i].window, "map window"))) return rc;
  }
  if ((rc = check_lightcurves(ctx, lcs))) return rc;
  if (!trajs) return fail(ctx, MORSE_EINVAL, "trajs is NULL");
  if (trajs->kind == MORSE_TRAJ_GRID) {
    if (trajs->n_u0 <= 0 || trajs->n_alpha <= 0 || trajs->n_t0 <= 0 || trajs->n_tE <= 0 ||
        !trajs->h_u0 || !trajs->h_alpha || !trajs->h_t0 || !trajs->h_tE)
      return fail(ctx, MORSE_EINVAL, "grid trajectories: empty axis or NULL array");
    for (int i = 0; i < trajs->n_tE; ++i)
      if (!(trajs->h_tE[i] > 0 && std::isfinite(trajs->h_tE[i])))
        return fail(ctx, MORSE_EINVAL, "grid trajectories: tE must be finite and > 0");
    for (int i = 0; i < trajs->n_u0; ++i)
      if (!std::isfinite(trajs->h_u0[i])) return fail(ctx, MORSE_EINVAL, "grid: u0 not finite");
    for (int i = 0; i < trajs->n_alpha; ++i)
      if (!std::isfinite(trajs->h_alpha[i])) return fail(ctx, MORSE_EINVAL, "grid: alpha not finite");
    for (int i = 0; i < trajs->n_t0; ++i)
      if (!std::isfinite(trajs->h_t0[i])) return fail(ctx, MORSE_EINVAL, "grid: t0 not finite");
  } else if (trajs->kind == MORSE_TRAJ_LIST) {
    if (trajs->n <= 0 || !trajs->d_params) return fail(ctx, MORSE_EINVAL, "list trajectories: n <= 0 or NULL");
  } else {
    return fail(ctx, MORSE_EINVAL, "unknown trajectory kind %d", trajs->kind);
  }
  return MORSE_OK;
}

int64_t traj_count(const morse_trajectories* t) {
  return t->kind == MORSE_TRAJ_GRID ? (int64_t)t->n_u0 * t->n_alpha * t->n_t0 * t->n_tE : t->n;
}

uint64_t metadata_key(const morse_map_view* maps, int32_t n_maps, const morse_lightcurves* lcs,
                      const morse_trajectories* trajs) {
  Hasher h;
  h.pod(n_maps);
  for (int i = 0; i < n_maps; ++i) {
    h.pod(maps[i].d_map);
    h.pod(maps[i].window);
  }
  h.pod(lcs->n_events);
  h.bytes(lcs->h_offsets, sizeof(int64_t) * (lcs->n_events + 1));
  h.bytes(lcs->h_t_ref, sizeof(double) * lcs->n_events);
  h.pod(trajs->kind);
  if (trajs->kind == MORSE_TRAJ_GRID) {
    h.pod(trajs->n_u0);
    h.pod(trajs->n_alpha);
    h.pod(trajs->n_t0);
    h.pod(trajs->n_tE);
    h.bytes(trajs->h_u0, 8 * trajs->n_u0);
    h.bytes(trajs->h_alpha, 8 * trajs->n_alpha);
    h.bytes(trajs->h_t0, 8 * trajs->n_t0);
    h.bytes(trajs->h_tE, 8 * trajs->n_tE);
  }
  return h.h;
}

// Reserve the workspace and upload the host metadata of a search into its own buffer
// (skipped when the same metadata is already resident).  Enqueues nothing else.
int plan_search(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                const morse_lightcurves* lcs, const morse_trajectories* trajs,
                const morse_search_out* out, SearchPlan& sp) {
  int rc;
  sp.n_traj = traj_count(trajs);
  sp.n_events = lcs->n_events;
  sp.n_maps = n_maps;
  sp.n_pts = lcs->h_offsets[lcs->n_events];
  const int64_t n_tc = (trajs->kind == MORSE_TRAJ_LIST && !trajs->shared)
                           ? sp.n_traj * lcs->n_events
                           : sp.n_traj;
  const int64_t n_out = (int64_t)sp.n_events * n_maps * sp.n_traj;
  const bool need_chi2 = !out->d_chi2 && (out->d_best_chi2 || out->d_best_idx || out->top_k > 0);
  const int32_t k = out->top_k;
  const int n_axes = trajs->kind == MORSE_TRAJ_GRID
                         ? trajs->n_u0 + trajs->n_alpha + trajs->n_t0 + trajs->n_tE
                         : 0;
  if ((rc = check_quad_size(ctx, maps, n_maps))) return rc;
  // lists are scored in an order grouped by direction (one counting sort per list)
  sp.perm_lists = (trajs->kind == MORSE_TRAJ_LIST && sp.n_traj > 0) ? (int32_t)(n_tc / sp.n_traj) : 0;
  if ((int64_t)sp.perm_lists * kPermBins > kPermBinsMax || n_tc > INT32_MAX) sp.perm_lists = 0;
  Plan pl;
  const size_t i_quad = pl.add(quad_region_bytes(maps, n_maps)),
               i_sums = pl.add(24 * (size_t)sp.n_events), i_cnt = pl.add(4 * kQueueWords),
               i_wF = pl.add(8 * (size_t)sp.n_pts), i_tc = pl.add(sizeof(TrajC) * (size_t)n_tc),
               i_chi = pl.add(need_chi2 ? 8 * (size_t)n_out : 0),
               i_tk = pl.add(k > 0 ? topk_scratch_bytes(sp.n_events, k) : 0),
               i_perm = pl.add(sp.perm_lists ? 4 * (size_t)n_tc : 0),
               i_pk = pl.add(sp.perm_lists ? 4 * (size_t)n_tc : 0),
               i_ph = pl.add(4 * (size_t)sp.perm_lists * kPermBins);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  if (sp.perm_lists) {
    sp.perm = (int32_t*)pl.ptr(ctx, i_perm);
    sp.perm_key = (uint32_t*)pl.ptr(ctx, i_pk);
    sp.perm_hist = (uint32_t*)pl.ptr(ctx, i_ph);
  }
  double* d_sums = (double*)pl.ptr(ctx, i_sums);
  sp.counter = (uint32_t*)pl.ptr(ctx, i_cnt);
  double* d_wF = (double*)pl.ptr(ctx, i_wF);
  sp.tc = (TrajC*)pl.ptr(ctx, i_tc);
  sp.chi2 = out->d_chi2 ? out->d_chi2 : (double*)pl.ptr(ctx, i_chi);
  sp.tk_scratch = pl.ptr(ctx, i_tk);
  sp.num_cu = ctx->num_cu;
  sp.h_maps.resize(n_maps);
  for (int i = 0; i < n_maps; ++i) sp.h_maps[i] = make_mapc(maps[i].d_map, maps[i].window);
  assign_quads(sp.h_maps, pl.ptr(ctx, i_quad));
  // metadata buffer: offsets | reference times | map table | grid axes
  const size_t b_off = (8 * (size_t)(sp.n_events + 1) + 255) & ~size_t(255);
  const size_t b_tref = (8 * (size_t)sp.n_events + 255) & ~size_t(255);
  const size_t b_maps = (sizeof(MapC) * n_maps + 255) & ~size_t(255);
  if ((rc = reserve_meta(ctx, ctx->smeta, b_off + b_tref + b_maps + 8 * (size_t)n_axes))) return rc;
  int64_t* d_off = (int64_t*)ctx->smeta.p;
  double* d_tref = (double*)(ctx->smeta.p + b_off);
  sp.d_maps = (MapC*)(ctx->smeta.p + b_off + b_tref);
  sp.axes = (double*)(ctx->smeta.p + b_off + b_tref + b_maps);
  Hasher key;
  key.pod(ctx->smeta.p);
  key.pod(metadata_key(maps, n_maps, lcs, trajs));
  key.bytes(sp.h_maps.data(), sizeof(MapC) * n_maps);  // includes the packed-cell addresses
  if (key.h != ctx->smeta.key) {
    ctx->smeta.key = 0;
    std::vector<double> axes;
    if (n_axes) {
      axes.insert(axes.end(), trajs->h_u0, trajs->h_u0 + trajs->n_u0);
      axes.insert(axes.end(), trajs->h_alpha, trajs->h_alpha + trajs->n_alpha);
      axes.insert(axes.end(), trajs->h_t0, trajs->h_t0 + trajs->n_t0);
      axes.insert(axes.end(), trajs->h_tE, trajs->h_tE + trajs->n_tE);
    }
    if ((rc = upload(ctx, d_off, lcs->h_offsets, 8 * (sp.n_events + 1)))) return rc;
    if ((rc = upload(ctx, d_tref, lcs->h_t_ref, 8 * sp.n_events))) return rc;
    if ((rc = upload(ctx, sp.d_maps, sp.h_maps.data(), sizeof(MapC) * n_maps))) return rc;
    if ((rc = upload(ctx, sp.axes, axes.data(), 8 * axes.size()))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // host arrays go out of scope
    ctx->smeta.key = key.h;
  }
  sp.lc.t = lcs->d_t;
  sp.lc.w = lcs->d_weight;
  sp.lc.F = lcs->d_flux;
  sp.lc.wFc = d_wF;
  sp.lc.off = d_off;
  sp.lc.sums = d_sums;
  sp.lc.t_ref = d_tref;
  return MORSE_OK;
}

// Preparation kernels (map packing, light-curve sums, trajectory constants).
hipError_t enqueue_prep(const SearchPlan& sp, const morse_trajectories* trajs, hipStream_t st) {
  hipError_t e = launch_quad_pack(sp.d_maps, sp.h_maps.data(), sp.n_maps, st);
  if (e != hipSuccess) return e;
  e = launch_lc_prep(sp.lc.t, sp.lc.F, sp.lc.w, sp.lc.off, sp.n_events,
                                (double*)sp.lc.wFc, (double*)sp.lc.sums, st);
  if (e != hipSuccess) return e;
  if (trajs->kind == MORSE_TRAJ_GRID)
    return launch_traj_prep_grid(sp.axes, trajs->n_u0, trajs->n_alpha, trajs->n_t0, trajs->n_tE,
                                 sp.tc, st);
  const int64_t n = trajs->shared ? sp.n_traj : sp.n_traj * sp.n_events;
  e = launch_traj_prep_list(trajs->d_params, n, sp.tc, st);
  if (e != hipSuccess || !sp.perm) return e;
  return launch_traj_perm(sp.tc, sp.n_traj, sp.perm_lists, sp.perm_key, sp.perm_hist, sp.perm, st);
}

hipError_t enqueue_select(const SearchPlan& sp, const morse_search_out* out, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (out->d_best_chi2 || out->d_best_idx)
    e = launch_best(sp.chi2, (int64_t)sp.n_events * sp.n_maps, sp.n_traj, out->d_best_chi2,
                    out->d_best_idx, st);
  if (e == hipSuccess && out->top_k > 0)
    e = launch_topk(sp.chi2, sp.n_events, (int64_t)sp.n_maps * sp.n_traj, out->top_k,
                    out->d_topk_chi2, out->d_topk_idx, sp.tk_scratch, sp.num_cu, st);
  return e;
}

BatchedArgs batched_args(morse_ctx* ctx, const SearchPlan& sp, const morse_trajectories* trajs,
                         const morse_search_out* out, const TuneCfg& cfg) {
  BatchedArgs a;
  a.tc = sp.tc;
  a.n_traj = sp.n_traj;
  a.shared = (trajs->kind == MORSE_TRAJ_GRID || trajs->shared) ? 1 : 0;
  a.n_events = sp.n_events;
  a.n_maps = sp.n_maps;
  a.maps = sp.d_maps;
  a.lc = sp.lc;
  a.out.chi2 = sp.chi2;
  a.out.fs = out->d_fs;
  a.out.fb = out->d_fb;
  a.counter = sp.counter;
  a.nu = a.na = a.nt = a.ne = 0;
  if (trajs->kind == MORSE_TRAJ_GRID) {
    a.nu = trajs->n_u0;
    a.na = trajs->n_alpha;
    a.nt = trajs->n_t0;
    a.ne = trajs->n_tE;
  }
  a.perm = sp.perm;
  a.traj_per_item = cfg.traj_per_item;
  a.waves_per_block = cfg.waves_per_block;
  a.tu = cfg.tu;
  const int64_t nb = (sp.n_traj + cfg.traj_per_item - 1) / cfg.traj_per_item;
  const int64_t items = nb * sp.n_events * sp.n_maps;
  int64_t blocks = (int64_t)ctx->num_cu * cfg.blocks_per_cu;
  const int64_t need = (items + cfg.waves_per_block - 1) / cfg.waves_per_block;
  if (blocks > need) blocks = need;
  a.grid_blocks = (int32_t)std::max<int64_t>(blocks, 1);
  return a;
}

// Reads an autotune cache ({"class": index, ...}); false when the file cannot be read.
bool read_tune_cache(const char* path, std::map<std::string, int>& all) {
  std::ifstream in(path);
  if (!in) return false;
  std::string txt((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
  size_t p = 0;
  while ((p = txt.find('"', p)) != std::string::npos) {
    size_t q = txt.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string k = txt.substr(p + 1, q - p - 1);
    size_t colon = txt.find(':', q);
    if (colon == std::string::npos) break;
    all[k] = std::atoi(txt.c_str() + colon + 1);
    p = txt.find_first_of(",}", colon);
    if (p == std::string::npos) break;
  }
  return true;
}

std::string shape_class(const SearchPlan& sp) {
  auto bucket = [](double v) { return (int)std::floor(std::log2(std::max(v, 1.0))); };
  std::ostringstream s;
  s << "gfx950|v3|maps" << bucket(sp.n_maps) << "|pts" << bucket((double)sp.n_pts / sp.n_events)
    << "|traj" << bucket((double)sp.n_traj) << "|ev" << bucket(sp.n_events);
  return s.str();
}

}  // namespace

extern "C" {


int morse_search(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                 const morse_lightcurves* lcs, const morse_trajectories* trajs, int32_t mode,
                 morse_search_out* out) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (!out) return fail(ctx, MORSE_EINVAL, "out is NULL");
  int rc;
  if ((rc = validate_search(ctx, maps, n_maps, lcs, trajs))) return rc;
  if (mode != MORSE_SEARCH_PLAIN && mode != MORSE_SEARCH_BATCHED)
    return fail(ctx, MORSE_EINVAL, "unknown search mode %d", mode);
  if (out->top_k < 0 || out->top_k > 4096)
    return fail(ctx, out->top_k < 0 ? MORSE_EINVAL : MORSE_EUNSUPPORTED, "top_k must be in [0, 4096]");
  if (out->top_k > 0 && (!out->d_topk_chi2 || !out->d_topk_idx))
    return fail(ctx, MORSE_EINVAL, "top_k > 0 needs d_topk_chi2 and d_topk_idx");
  if (out->top_k > 0 && ((double)n_maps * (double)traj_count(trajs) >= 4294967295.0 ||
                         lcs->n_events > 65535))
    return fail(ctx, MORSE_ERANGE, "top-k needs n_maps * n_traj < 2^32 and at most 65535 events");
  {
    const int64_t nt = traj_count(trajs);
    if ((double)nt * lcs->n_events * n_maps >= 9.0e18 ||
        (double)nt * lcs->n_events * n_maps >= 2147483647.0)
      return fail(ctx, MORSE_ERANGE, "too many (event, map, trajectory) items");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  SearchPlan sp;
  if ((rc = plan_search(ctx, maps, n_maps, lcs, trajs, out, sp))) return rc;

  if (mode == MORSE_SEARCH_PLAIN) {
    HIP_TRY(ctx, enqueue_prep(sp, trajs, ctx->stream));
    for (int32_t e = 0; e < sp.n_events; ++e) {
      const TrajC* tc = sp.tc + ((trajs->kind == MORSE_TRAJ_LIST && !trajs->shared) ? (int64_t)e * sp.n_traj : 0);
      for (int32_t m = 0; m < n_maps; ++m) {
        const int64_t base = ((int64_t)e * n_maps + m) * sp.n_traj;
        SearchOut so{sp.chi2 + base, out->d_fs ? out->d_fs + base : nullptr,
                     out->d_fb ? out->d_fb + base : nullptr};
        LaunchTimer tm{ctx, MORSE_KERNEL_SEARCH};
        HIP_TRY(ctx, tm.begin(ctx->stream));
        HIP_TRY(ctx, launch_search_plain(tc, sp.n_traj, sp.lc, e, sp.h_maps[m], so, 4, ctx->stream));
        HIP_TRY(ctx, tm.end(ctx->stream));
      }
    }
    HIP_TRY(ctx, enqueue_select(sp, out, ctx->stream));
    return MORSE_OK;
  }

  // batched: one persistent launch, captured into a graph per argument set
  auto it = ctx->tune.find(shape_class(sp));
  const int cfg_idx = it == ctx->tune.end() ? 0 : it->second;
  const TuneCfg& cfg = kTune[cfg_idx];
  Hasher h;
  h.pod(metadata_key(maps, n_maps, lcs, trajs));
  h.pod(ctx->smeta.p);
  h.pod(ctx->ws_epoch);
  h.pod(cfg_idx);
  h.pod(*out);
  h.pod(lcs->d_t);
  h.pod(lcs->d_flux);
  h.pod(lcs->d_weight);
  h.pod(trajs->d_params);
  h.pod(trajs->shared);
  h.pod(trajs->n);
  if (timed(ctx, MORSE_KERNEL_SEARCH)) {  // same kernels, launched one by one
    const BatchedArgs a = batched_args(ctx, sp, trajs, out, cfg);
    HIP_TRY(ctx, enqueue_prep(sp, trajs, ctx->stream));
    HIP_TRY(ctx, launch_fill_u32(sp.counter, kQueueWords, 0u, ctx->stream));
    LaunchTimer tm{ctx, MORSE_KERNEL_SEARCH};
    HIP_TRY(ctx, tm.begin(ctx->stream));
    HIP_TRY(ctx, launch_search_batched(a, ctx->stream));
    HIP_TRY(ctx, tm.end(ctx->stream));
    HIP_TRY(ctx, enqueue_select(sp, out, ctx->stream));
    return MORSE_OK;
  }
  if (!ctx->gexec || ctx->graph_key != h.h) {
    if (ctx->gexec) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      (void)hipGraphExecDestroy(ctx->gexec);
      ctx->gexec = nullptr;
    }
    const BatchedArgs a = batched_args(ctx, sp, trajs, out, cfg);
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_prep(sp, trajs, ctx->capture_stream);
    if (e == hipSuccess) e = launch_fill_u32(sp.counter, kQueueWords, 0u, ctx->capture_stream);
    if (e == hipSuccess) e = launch_search_batched(a, ctx->capture_stream);
    if (e == hipSuccess) e = enqueue_select(sp, out, ctx->capture_stream);
    hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(ctx, MORSE_EHIP, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ctx->gexec = nullptr;
      return fail(ctx, MORSE_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    ctx->graph_key = h.h;
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
  return MORSE_OK;
}

int morse_autotune(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                   const morse_lightcurves* lcs, const morse_trajectories* trajs,
                   const char* cache_path, int32_t* h_best_config) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = validate_search(ctx, maps, n_maps, lcs, trajs))) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  morse_search_out out{};
  SearchPlan sp;
  if ((rc = plan_search(ctx, maps, n_maps, lcs, trajs, &out, sp))) return rc;
  const std::string cls = shape_class(sp);
  // time each candidate on (at most) the first 16 events x 8 maps of the problem
  SearchPlan sub = sp;
  sub.n_events = std::min(sp.n_events, 16);
  sub.n_maps = std::min(sp.n_maps, 8);
  const size_t need = (size_t)sub.n_events * sub.n_maps * sp.n_traj * 8;
  double* scratch = nullptr;
  HIP_TRY(ctx, hipMalloc((void**)&scratch, need));
  sub.chi2 = scratch;
  hipError_t e = enqueue_prep(sp, trajs, ctx->stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = 0;
  float best_ms = 1e30f;
  for (int c = 0; c < kNumTune && e == hipSuccess; ++c) {
    const BatchedArgs a = batched_args(ctx, sub, trajs, &out, kTune[c]);
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = launch_fill_u32(sub.counter, kQueueWords, 0u, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
      if (e == hipSuccess) e = launch_search_batched(a, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(ctx, MORSE_EHIP, "autotune: %s", hipGetErrorString(e));
  ctx->tune[cls] = best;
  if (h_best_config) *h_best_config = best;
  if (cache_path) {
    // JSON object {"class": index, ...}: merge with the existing file
    std::map<std::string, int> all;
    read_tune_cache(cache_path, all);
    all[cls] = best;
    std::ofstream o(cache_path);
    o << "{";
    bool first = true;
    for (auto& kv : all) {
      o << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
      first = false;
    }
    o << "}\n";
  }
  return MORSE_OK;
}

int morse_autotune_load(morse_ctx* ctx, const char* cache_path, int32_t* h_loaded) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (!cache_path) return fail(ctx, MORSE_EINVAL, "cache_path is NULL");
  std::map<std::string, int> all;
  if (!read_tune_cache(cache_path, all))
    return fail(ctx, MORSE_EUNSUPPORTED, "cannot read autotune cache %s", cache_path);
  int32_t n = 0;
  for (const auto& kv : all) {
    if (kv.second < 0 || kv.second >= kNumTune) continue;
    ctx->tune[kv.first] = kv.second;
    ++n;
  }
  if (h_loaded) *h_loaded = n;
  return MORSE_OK;
}

int morse_candidates_from_topk(morse_ctx* ctx, const morse_trajectories* trajs, int32_t n_events,
                               int32_t n_maps, int32_t top_k, const int64_t* d_topk_idx,
                               double* d_params, int32_t* d_event, int32_t* d_map_index) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (!trajs) return fail(ctx, MORSE_EINVAL, "trajs is NULL");
  if (n_events <= 0 || n_maps <= 0 || top_k <= 0)
    return fail(ctx, MORSE_EINVAL, "n_events, n_maps and top_k must be >= 1");
  if (!d_topk_idx || !d_params || !d_event || !d_map_index)
    return fail(ctx, MORSE_EINVAL, "NULL device pointer");
  const int64_t n_traj = traj_count(trajs);
  if (n_traj <= 0) return fail(ctx, MORSE_EINVAL, "empty trajectory set");
  if (trajs->kind == MORSE_TRAJ_LIST && !trajs->d_params)
    return fail(ctx, MORSE_EINVAL, "list trajectories: d_params is NULL");
  if (trajs->kind == MORSE_TRAJ_GRID &&
      (!trajs->h_u0 || !trajs->h_alpha || !trajs->h_t0 || !trajs->h_tE))
    return fail(ctx, MORSE_EINVAL, "grid trajectories: NULL axis");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double* axes = nullptr;
  int rc;
  if (trajs->kind == MORSE_TRAJ_GRID) {
    std::vector<double> h;
    h.insert(h.end(), trajs->h_u0, trajs->h_u0 + trajs->n_u0);
    h.insert(h.end(), trajs->h_alpha, trajs->h_alpha + trajs->n_alpha);
    h.insert(h.end(), trajs->h_t0, trajs->h_t0 + trajs->n_t0);
    h.insert(h.end(), trajs->h_tE, trajs->h_tE + trajs->n_tE);
    // the auxiliary buffer keeps the search's resident workspace intact
    if ((rc = reserve_aux(ctx, 8 * h.size()))) return rc;
    double* d = (double*)ctx->aux;
    if ((rc = upload(ctx, d, h.data(), 8 * h.size()))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    axes = d;
  }
  HIP_TRY(ctx, launch_candidates(axes, trajs->n_u0, trajs->n_alpha, trajs->n_t0, trajs->n_tE,
                                 trajs->d_params, trajs->shared, n_traj, n_events, n_maps, top_k,
                                 d_topk_idx, d_params, d_event, d_map_index, ctx->stream));
  return MORSE_OK;
}

}  // extern "C"
