// Host-side helpers shared by the C ABI's source files (api_*.hip): the context
// structure behind the opaque morse_ctx, error reporting, workspace and metadata
// buffers, argument validation and map descriptors.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "stack.h"
#include "lines.h"
#include "simplex.h"


// A device buffer of host metadata with the key of what it holds.
struct MetaBuf {
  char* p = nullptr;
  size_t size = 0;
  uint64_t key = 0;
};

struct morse_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t capture_stream = nullptr;  // private stream for graph capture
  hipStream_t fork_stream = nullptr;     // second chain of a refinement
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int num_cu = 256;
  char* ws = nullptr;
  size_t ws_size = 0;
  uint64_t ws_epoch = 0;  // bumps when the workspace moves
  std::string err;
  // host metadata of the searches and of the candidate entry points, each in a device
  // buffer of its own (never in the shared workspace, which the other entry points
  // overwrite) and uploaded only when its key changes
  MetaBuf smeta, cmeta;
  // source-radius stacks: direct-sum taps, FFT twiddle tables and the transforms of
  // the profile pairs, each kept until a call needs different ones
  MetaBuf stack_taps, fft_tw, fft_spec;
  // the packed-map descriptor of the line filter
  MetaBuf lmeta;
  // critical points and their caustic images of the last finite-source call (key: s, q,
  // phases)
  MetaBuf fs_crit;
  // split of the last stack call's radii (key of its arguments): direct radii with
  // their tap counts (taps in stack_taps, in this order), FFT radii, widest FFT stencil
  struct StackSplit {
    uint64_t key = 0;
    std::vector<int> direct_k, fft_k;
    std::vector<int32_t> ntaps;
    std::vector<int32_t> reach;  // per direct radius: the largest |offset| along x, then y
    size_t w_bytes = 0;  // the tap offsets follow the weights at this byte offset
    int rmx = 0, rmy = 0;
  } stack_split;
  // batched-search graph
  hipGraphExec_t gexec = nullptr;
  uint64_t graph_key = 0;
  // refinement graph
  hipGraphExec_t refine_gexec = nullptr;
  uint64_t refine_key = 0;
  // autotune choices per shape class
  std::map<std::string, int> tune;
  // small auxiliary device buffer, separate from the workspace
  char* aux = nullptr;
  size_t aux_size = 0;
  // disk-convolution taps resident on the device (key of the taps they hold)
  char* taps = nullptr;
  size_t taps_size = 0;
  uint64_t taps_key = 0;
  int32_t taps_n = 0;
  int32_t taps_rx = 0, taps_ry = 0;  // the largest |offset| of the taps along x and y
  size_t taps_wbytes = 0;
  // kernel timing: enabled families, pending event pairs, free events, totals
  uint32_t timing_mask = 0;
  struct Timed {
    int32_t kernel;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> free_events;
  double time_ms[3] = {0.0, 0.0, 0.0};
  int64_t launches[3] = {0, 0, 0};
};

namespace morse {
namespace host {

// Message of the last error of this thread (returned by morse_last_error(NULL)).
extern thread_local std::string g_thread_error;


inline int fail(morse_ctx* ctx, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  g_thread_error = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((ctx), MORSE_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// FNV-1a over raw bytes, for keys of uploaded metadata and captured graphs.
struct Hasher {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  }
  template <class T>
  void pod(const T& v) {
    bytes(&v, sizeof(T));
  }
};

// Folds the pending timing events into the totals (waits for them).
inline hipError_t resolve_timers(morse_ctx* ctx) {
  for (const auto& t : ctx->timed) {
    hipError_t e = hipEventSynchronize(t.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return e;
    ctx->time_ms[t.kernel] += ms;
    ctx->launches[t.kernel] += 1;
    ctx->free_events.push_back(t.a);
    ctx->free_events.push_back(t.b);
  }
  ctx->timed.clear();
  return hipSuccess;
}

inline hipError_t take_event(morse_ctx* ctx, hipEvent_t* e) {
  if (!ctx->free_events.empty()) {
    *e = ctx->free_events.back();
    ctx->free_events.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

inline bool timed(const morse_ctx* ctx, int32_t kernel) { return (ctx->timing_mask >> kernel) & 1u; }

// Brackets one launch of a kernel family with events on `st` when the family is timed.
struct LaunchTimer {
  morse_ctx* ctx;
  int32_t kernel;
  hipEvent_t a = nullptr;
  hipError_t begin(hipStream_t st) {
    if (!timed(ctx, kernel)) return hipSuccess;
    hipError_t e = take_event(ctx, &a);
    return e == hipSuccess ? hipEventRecord(a, st) : e;
  }
  hipError_t end(hipStream_t st) {
    if (!a) return hipSuccess;
    hipEvent_t b = nullptr;
    hipError_t e = take_event(ctx, &b);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    ctx->timed.push_back({kernel, a, b});
    a = nullptr;
    // bound the pending list for callers that never read the totals
    return ctx->timed.size() >= 4096 ? resolve_timers(ctx) : hipSuccess;
  }
};

// Bump allocator over the context workspace: first collect sizes, then reserve.
struct Plan {
  std::vector<size_t> sizes;
  size_t add(size_t bytes) {
    sizes.push_back((bytes + 255) & ~size_t(255));
    return sizes.size() - 1;
  }
  size_t total() const {
    size_t t = 0;
    for (size_t s : sizes) t += s;
    return t;
  }
  char* ptr(morse_ctx* ctx, size_t id) const { return ptr_at(ctx->ws, id); }
  char* ptr_at(char* base, size_t id) const {
    size_t off = 0;
    for (size_t i = 0; i < id; ++i) off += sizes[i];
    return base + off;
  }
};

inline int reserve(morse_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return MORSE_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->gexec) {
    (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    ctx->graph_key = 0;
  }
  if (ctx->refine_gexec) {
    (void)hipGraphExecDestroy(ctx->refine_gexec);
    ctx->refine_gexec = nullptr;
    ctx->refine_key = 0;
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_size = 0;
  size_t want = std::max(bytes, size_t(1) << 20);
  want = (want + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
  if (hipMalloc((void**)&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, MORSE_ENOMEM, "workspace allocation of %zu bytes failed", want);
  }
  ctx->ws_size = want;
  ctx->ws_epoch++;
  return MORSE_OK;
}

inline int reserve_aux(morse_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->aux_size) return MORSE_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->aux) (void)hipFree(ctx->aux);
  ctx->aux = nullptr;
  ctx->aux_size = 0;
  const size_t want = std::max(bytes, size_t(1) << 16);
  if (hipMalloc((void**)&ctx->aux, want) != hipSuccess) {
    ctx->aux = nullptr;
    return fail(ctx, MORSE_ENOMEM, "auxiliary allocation of %zu bytes failed", want);
  }
  ctx->aux_size = want;
  return MORSE_OK;
}

// The largest |offset| along x and along y of a tap table (pairs dx, dy).
inline void tap_reach(const std::vector<int32_t>& off, int32_t& rx, int32_t& ry) {
  rx = ry = 0;
  for (size_t k = 0; k + 1 < off.size(); k += 2) {
    rx = std::max(rx, std::abs(off[k]));
    ry = std::max(ry, std::abs(off[k + 1]));
  }
}

// Grows a metadata buffer to at least `bytes` (its contents are then invalid).
inline int reserve_meta(morse_ctx* ctx, MetaBuf& mb, size_t bytes) {
  if (bytes <= mb.size) return MORSE_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (mb.p) (void)hipFree(mb.p);
  mb.p = nullptr;
  mb.size = 0;
  mb.key = 0;
  if (hipMalloc((void**)&mb.p, bytes) != hipSuccess) {
    mb.p = nullptr;
    return fail(ctx, MORSE_ENOMEM, "metadata allocation of %zu bytes failed", bytes);
  }
  mb.size = bytes;
  return MORSE_OK;
}

inline int upload(morse_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (!bytes) return MORSE_OK;
  HIP_TRY(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  return MORSE_OK;
}

inline bool grid_ok(const morse_grid2d* g) {
  return g && std::isfinite(g->cx) && std::isfinite(g->cy) && std::isfinite(g->wx) &&
         std::isfinite(g->wy) && g->wx > 0 && g->wy > 0 && g->nx >= 2 && g->ny >= 2 &&
         (g->nx % 2) == 0 && (g->ny % 2) == 0;
}

inline int check_lens(morse_ctx* ctx, double s, double q) {
  if (!(std::isfinite(s) && s > 0)) return fail(ctx, MORSE_EINVAL, "s must be finite and > 0");
  if (!(q >= 0.0 && q <= 1.0)) return fail(ctx, MORSE_EINVAL, "q must lie in [0, 1]");
  return MORSE_OK;
}

inline int check_window(morse_ctx* ctx, const morse_grid2d* w, const char* what) {
  if (!grid_ok(w)) return fail(ctx, MORSE_EINVAL, "%s: invalid grid (even counts >= 2, finite widths > 0)", what);
  if (w->nx > 32768 || w->ny > 32768)
    return fail(ctx, MORSE_ERANGE, "%s: at most 32768 pixels per side", what);
  return MORSE_OK;
}

inline MapC make_mapc(const float* map, const morse_grid2d& w) {
  MapC m;
  m.map = map;
  m.mx = w.nx;
  m.my = w.ny;
  m.sx = (float)w.cx;
  m.sy = (float)w.cy;
  m.kx = (float)((double)w.nx / w.wx);
  m.ky = (float)((double)w.ny / w.wy);
  m.ox = (float)(w.nx / 2) - 0.5f;
  m.oy = (float)(w.ny / 2) - 0.5f;
  m.lx = (float)(w.nx - 1);
  m.ly = (float)(w.ny - 1);
  m.tiles_x = (uint32_t)((w.nx - 1 + 3) / 4);
  m.tiles_y = (uint32_t)((w.ny - 1 + 1) / 2);
  m.quad = nullptr;
  return m;
}

// Quad-packed maps live in one workspace region: per map quad_bytes rounded to 256.
inline size_t quad_region_bytes(const morse_map_view* maps, int32_t n_maps) {
  size_t t = 0;
  for (int i = 0; i < n_maps; ++i)
    t += (quad_bytes(maps[i].window.nx, maps[i].window.ny) + 255) & ~size_t(255);
  return t;
}

inline void assign_quads(std::vector<MapC>& hm, char* region) {
  for (auto& m : hm) {
    m.quad = (const Quad*)region;
    region += (quad_bytes(m.mx, m.my) + 255) & ~size_t(255);
  }
}

// Critical points of the binary lens at nphi equally spaced phases of the critical-curve
// quartic (4 per phase, phase-major; defined with the caustic geometry).
void critical_points(double s, double q, int32_t nphi, std::vector<std::complex<double>>& z);

// Device address of the allocation-free entry point's scratch array on `device`
// (looked up once per device, with that device current; defined beside the entry
// point).  Returns MORSE_OK and sets *out, or an error code.
int noalloc_scratch(int device, char** out);

// Light curves: arrays present, CSR offsets from 0, each event at least 3 and at most
// kMaxEventPoints points (the kernels address an event's FP64 arrays with 32-bit byte
// offsets from the event's base, 8 B x 2^28 < 2^32), finite reference times.
constexpr int64_t kMaxEventPoints = (int64_t)1 << 28;

inline int check_lightcurves(morse_ctx* ctx, const morse_lightcurves* lcs) {
  if (!lcs || lcs->n_events <= 0 || !lcs->h_offsets || !lcs->h_t_ref || !lcs->d_t || !lcs->d_flux ||
      !lcs->d_weight)
    return fail(ctx, MORSE_EINVAL, "light curves: missing arrays or n_events <= 0");
  if (lcs->h_offsets[0] != 0) return fail(ctx, MORSE_EINVAL, "light curves: offsets[0] must be 0");
  for (int e = 0; e < lcs->n_events; ++e) {
    const int64_t n = lcs->h_offsets[e + 1] - lcs->h_offsets[e];
    if (n < 3) return fail(ctx, MORSE_EINVAL, "event %d has %lld < 3 points", e, (long long)n);
    if (n > kMaxEventPoints)
      return fail(ctx, MORSE_ERANGE, "event %d has %lld points, more than 2^28", e, (long long)n);
    if (!std::isfinite(lcs->h_t_ref[e])) return fail(ctx, MORSE_EINVAL, "event %d: t_ref not finite", e);
  }
  return MORSE_OK;
}

inline int check_quad_size(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps) {
  for (int i = 0; i < n_maps; ++i)
    if (quad_bytes(maps[i].window.nx, maps[i].window.ny) >= ((size_t)1 << 32))
      return fail(ctx, MORSE_ERANGE, "map %d: %d x %d pixels exceed the 4 GiB packed-cell limit", i,
                  maps[i].window.nx, maps[i].window.ny);
  return MORSE_OK;
}


}  // namespace host
}  // namespace morse
