// C ABI of the gfx950 map-build / trajectory-search library (declared in
// include/morse.h): context and workspace management, host-side validation, the
// small host preparations (binary32 constants, disk-overlap weights) and the launch
// sequences of each entry point.  Every numerical step of the path runs in the HIP
// kernels of maps.hip, search.hip and refine.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "stack.h"
#include "lines.h"
#include "simplex.h"

using namespace morse;

namespace {

thread_local std::string g_thread_error;

struct TuneCfg {
  int traj_per_item;
  int waves_per_block;
  int blocks_per_cu;
  int tu;
};
// Candidate shapes of the batched search tried by the autotuner; index 0 is the
// default before tuning.  traj_per_item = trajectories per wavefront work item,
// tu = trajectories scored together by one wavefront (sharing light-curve loads).
const TuneCfg kTune[] = {
    {8, 4, 16, 2},  {8, 4, 16, 1},  {16, 4, 16, 2}, {8, 8, 8, 2},
    {32, 8, 8, 2},  {4, 4, 16, 2},  {16, 8, 4, 4},  {8, 2, 32, 2},
    {16, 4, 16, 4}, {32, 8, 8, 1},  {8, 2, 32, 1},  {64, 4, 8, 4},
    {32, 8, 4, 4},  {16, 4, 8, 4},  {8, 8, 4, 4},   {16, 8, 2, 4},
};
constexpr int kNumTune = sizeof(kTune) / sizeof(kTune[0]);

}  // namespace

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
  // split of the last stack call's radii (key of its arguments): direct radii with
  // their tap counts (taps in stack_taps, in this order), FFT radii, widest FFT stencil
  struct StackSplit {
    uint64_t key = 0;
    std::vector<int> direct_k, fft_k;
    std::vector<int32_t> ntaps;
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

namespace {

int fail(morse_ctx* ctx, int code, const char* fmt, ...) {
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
hipError_t resolve_timers(morse_ctx* ctx) {
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

hipError_t take_event(morse_ctx* ctx, hipEvent_t* e) {
  if (!ctx->free_events.empty()) {
    *e = ctx->free_events.back();
    ctx->free_events.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

bool timed(const morse_ctx* ctx, int32_t kernel) { return (ctx->timing_mask >> kernel) & 1u; }

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
  char* ptr(morse_ctx* ctx, size_t id) const {
    size_t off = 0;
    for (size_t i = 0; i < id; ++i) off += sizes[i];
    return ctx->ws + off;
  }
};

int reserve(morse_ctx* ctx, size_t bytes) {
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

int reserve_aux(morse_ctx* ctx, size_t bytes) {
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

// Grows a metadata buffer to at least `bytes` (its contents are then invalid).
int reserve_meta(morse_ctx* ctx, MetaBuf& mb, size_t bytes) {
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

int upload(morse_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (!bytes) return MORSE_OK;
  HIP_TRY(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  return MORSE_OK;
}

bool grid_ok(const morse_grid2d* g) {
  return g && std::isfinite(g->cx) && std::isfinite(g->cy) && std::isfinite(g->wx) &&
         std::isfinite(g->wy) && g->wx > 0 && g->wy > 0 && g->nx >= 2 && g->ny >= 2 &&
         (g->nx % 2) == 0 && (g->ny % 2) == 0;
}

int check_lens(morse_ctx* ctx, double s, double q) {
  if (!(std::isfinite(s) && s > 0)) return fail(ctx, MORSE_EINVAL, "s must be finite and > 0");
  if (!(q >= 0.0 && q <= 1.0)) return fail(ctx, MORSE_EINVAL, "q must lie in [0, 1]");
  return MORSE_OK;
}

int check_window(morse_ctx* ctx, const morse_grid2d* w, const char* what) {
  if (!grid_ok(w)) return fail(ctx, MORSE_EINVAL, "%s: invalid grid (even counts >= 2, finite widths > 0)", what);
  if (w->nx > 32768 || w->ny > 32768)
    return fail(ctx, MORSE_ERANGE, "%s: at most 32768 pixels per side", what);
  return MORSE_OK;
}

MapC make_mapc(const float* map, const morse_grid2d& w) {
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
size_t quad_region_bytes(const morse_map_view* maps, int32_t n_maps) {
  size_t t = 0;
  for (int i = 0; i < n_maps; ++i)
    t += (quad_bytes(maps[i].window.nx, maps[i].window.ny) + 255) & ~size_t(255);
  return t;
}

void assign_quads(std::vector<MapC>& hm, char* region) {
  for (auto& m : hm) {
    m.quad = (const Quad*)region;
    region += (quad_bytes(m.mx, m.my) + 255) & ~size_t(255);
  }
}

int check_quad_size(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps) {
  for (int i = 0; i < n_maps; ++i)
    if (quad_bytes(maps[i].window.nx, maps[i].window.ny) >= ((size_t)1 << 32))
      return fail(ctx, MORSE_ERANGE, "map %d: %d x %d pixels exceed the 4 GiB packed-cell limit", i,
                  maps[i].window.nx, maps[i].window.ny);
  return MORSE_OK;
}

// ---------------------------------------------------------------------------
// Uniform-disk / pixel overlap weights.  Area of disk(0, R) ∩ [x1,x2] x [y1,y2] as
// the integral over x of the chord length clipped to [y1, y2]; with x = R sin(th)
// the chord half-length is R cos(th) and the integrand is smooth between the angles
// where the clipped chord changes form, so each piece is integrated by 24-point
// Gauss-Legendre (nodes by Newton iteration on the Legendre polynomial).
struct Gauss {
  double x[24], w[24];
  Gauss() {
    const int n = 24;
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        double dp = n * (z * p1 - p0) / (z * z - 1.0);
        double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

double chord_clip(double R, double th, double y1, double y2) {
  double h = R * std::cos(th);
  double top = std::min(y2, h), bot = std::max(y1, -h);
  return top > bot ? top - bot : 0.0;
}

double rect_disk_area(double R, double x1, double x2, double y1, double y2) {
  static const Gauss G;
  double a = std::max(x1, -R), b = std::min(x2, R);
  if (!(b > a)) return 0.0;
  double ta = std::asin(a / R), tb = std::asin(b / R);
  std::vector<double> cuts = {ta, tb};
  for (double y : {y1, y2})
    if (std::fabs(y) < R) {
      double c = std::acos(std::fabs(y) / R);
      for (double th : {c, -c})
        if (th > ta && th < tb) cuts.push_back(th);
    }
  std::sort(cuts.begin(), cuts.end());
  double area = 0.0;
  for (size_t k = 0; k + 1 < cuts.size(); ++k) {
    double lo = cuts[k], hi = cuts[k + 1];
    double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    for (int i = 0; i < 24; ++i) {
      double th = mid + half * G.x[i];
      area += half * G.w[i] * chord_clip(R, th, y1, y2) * R * std::cos(th);
    }
  }
  return area;
}

// Volume under the unit hemisphere z = sqrt(1 - X^2 - Y^2) over {X >= a, Y >= b}.
// For a, b >= 0 inside the disk, integrating over Y in closed form and then by parts
// over X gives
//   (pi/2 - atan(a b / r))/3 + a b r/3 - b (3 - b^2)/6 acos(a / sqrt(1 - b^2))
//     - a (3 - a^2)/6 acos(b / sqrt(1 - a^2)),   r = sqrt(1 - a^2 - b^2);
// negative a or b follow by reflection from the half-space volume
// H(t) = pi (2 - 3t + t^3)/6 over {X >= t}.
double hemi_half(double t) {
  if (t <= -1.0) return 2.0 * M_PI / 3.0;
  if (t >= 1.0) return 0.0;
  return M_PI / 6.0 * (2.0 - 3.0 * t + t * t * t);
}

double hemi_upper(double a, double b) {
  if (a < 0.0) return hemi_half(b) - hemi_upper(-a, b);
  if (b < 0.0) return hemi_half(a) - hemi_upper(a, -b);
  const double s2 = a * a + b * b;
  if (s2 >= 1.0) return 0.0;
  const double r = std::sqrt(1.0 - s2);
  const double ca = std::min(1.0, a / std::sqrt(1.0 - b * b));
  const double cb = std::min(1.0, b / std::sqrt(1.0 - a * a));
  return (0.5 * M_PI - std::atan2(a * b, r)) / 3.0 + a * b * r / 3.0 -
         b * (3.0 - b * b) / 6.0 * std::acos(ca) - a * (3.0 - a * a) / 6.0 * std::acos(cb);
}

// Integral of sqrt(R^2 - x^2 - y^2) over disk(0, R) ∩ [x1,x2] x [y1,y2].
double rect_hemi_volume(double R, double x1, double x2, double y1, double y2) {
  const double u1 = x1 / R, u2 = x2 / R, v1 = y1 / R, v2 = y2 / R;
  const double v = hemi_upper(u1, v1) - hemi_upper(u2, v1) - hemi_upper(u1, v2) + hemi_upper(u2, v2);
  return std::max(0.0, v) * R * R * R;
}

// Unnormalised weight of the pixel at offset (a, b) for the limb-darkened disk of
// radius rho: the integral over pixel ∩ disk of I(r) = 1 - gamma (1 - 1.5 sqrt(1 -
// r^2/rho^2)), i.e. (1 - gamma) area + 1.5 gamma/rho volume.  gamma = 0 gives the area
// term alone (the uniform disk).
double profile_pixel(double rho, double dx, double dy, double gamma, int a, int b) {
  const double nx = std::max(0.0, (std::abs(a) - 0.5) * dx), ny = std::max(0.0, (std::abs(b) - 0.5) * dy);
  if (nx * nx + ny * ny >= rho * rho) return 0.0;  // the pixel does not meet the disk
  const double fx = (std::abs(a) + 0.5) * dx, fy = (std::abs(b) + 0.5) * dy;
  const double x1 = (a - 0.5) * dx, x2 = (a + 0.5) * dx, y1 = (b - 0.5) * dy, y2 = (b + 0.5) * dy;
  const double area = (fx * fx + fy * fy <= rho * rho) ? dx * dy : rect_disk_area(rho, x1, x2, y1, y2);
  if (gamma == 0.0) return area;
  return (1.0 - gamma) * area + 1.5 * gamma / rho * rect_hemi_volume(rho, x1, x2, y1, y2);
}

int stencil_half(double rho, double d) { return rho > 0.0 ? (int)std::ceil(rho / d + 0.5) : 0; }

// Taps (dx, dy offsets and binary32 weights), row-major over the stencil, zero taps
// dropped, weights normalised to sum 1 in FP64 and rounded once; rho within half a
// pixel gives the single tap 1.  Limited to stencils of at most 31 x 31.
int profile_taps(morse_ctx* ctx, double rho, double dx, double dy, double gamma,
                 std::vector<float>& w, std::vector<int32_t>& off) {
  w.clear();
  off.clear();
  if (rho <= 0.0) {
    w.push_back(1.0f);
    off.push_back(0);
    off.push_back(0);
    return MORSE_OK;
  }
  const int Rx = stencil_half(rho, dx), Ry = stencil_half(rho, dy);
  if (Rx > 15 || Ry > 15)
    return fail(ctx, MORSE_ERANGE, "disk radius spans more than 15 pixels (stencil > 31)");
  std::vector<double> wd;
  std::vector<int32_t> od;
  double sum = 0.0;
  for (int b = -Ry; b <= Ry; ++b)
    for (int a = -Rx; a <= Rx; ++a) {
      const double v = profile_pixel(rho, dx, dy, gamma, a, b);
      wd.push_back(v);
      od.push_back(a);
      od.push_back(b);
      sum += v;
    }
  for (size_t k = 0; k < wd.size(); ++k) {
    if (wd[k] == 0.0) continue;
    w.push_back((float)(wd[k] / sum));
    off.push_back(od[2 * k]);
    off.push_back(od[2 * k + 1]);
  }
  return MORSE_OK;
}

int disk_taps(morse_ctx* ctx, double rho, double dx, double dy, std::vector<float>& w,
              std::vector<int32_t>& off) {
  return profile_taps(ctx, rho, dx, dy, 0.0, w, off);
}

// FP64 quadrant q[b][a] (0 <= a <= Rx, 0 <= b <= Ry) of the weights normalised to sum
// 1 over the whole stencil (the weights are even in a and in b).
void profile_quadrant(double rho, double dx, double dy, double gamma, int Rx, int Ry,
                      std::vector<double>& q) {
  q.assign((size_t)(Rx + 1) * (Ry + 1), 0.0);
  double sum = 0.0;
  for (int b = 0; b <= Ry; ++b)
    for (int a = 0; a <= Rx; ++a) {
      const double v = profile_pixel(rho, dx, dy, gamma, a, b);
      q[(size_t)b * (Rx + 1) + a] = v;
      sum += v * (a ? 2.0 : 1.0) * (b ? 2.0 : 1.0);
    }
  for (double& v : q) v /= sum;
}


// Roots of the quartic c[0] + c[1] z + ... + c[4] z^4 by the Aberth-Ehrlich iteration
// (simultaneous Newton steps corrected by the other roots' repulsion), started from z
// when warm (continuation along the phase) or from a circle, then two Newton steps.
void quartic_roots(const std::complex<double> (&c)[5], std::complex<double> (&z)[4], bool warm) {
  typedef std::complex<double> C;
  auto p = [&](C x) { return (((c[4] * x + c[3]) * x + c[2]) * x + c[1]) * x + c[0]; };
  auto dp = [&](C x) { return ((4.0 * c[4] * x + 3.0 * c[3]) * x + 2.0 * c[2]) * x + c[1]; };
  if (!warm) {
    double rad = 0.0;
    for (int i = 0; i < 4; ++i) rad = std::max(rad, std::abs(c[i] / c[4]));
    rad = 1.0 + rad;
    for (int k = 0; k < 4; ++k) z[k] = std::polar(rad, 0.4 + 2.0 * M_PI * k / 4.0);
  }
  for (int it = 0; it < 500; ++it) {
    double moved = 0.0;
    for (int k = 0; k < 4; ++k) {
      const C pk = p(z[k]), dk = dp(z[k]);
      if (pk == 0.0) continue;
      const C ratio = pk / dk;
      C rep = 0.0;
      for (int j = 0; j < 4; ++j)
        if (j != k) rep += 1.0 / (z[k] - z[j]);
      const C step = ratio / (1.0 - ratio * rep);
      z[k] -= step;
      moved = std::max(moved, std::abs(step) / (1.0 + std::abs(z[k])));
    }
    if (moved < 1e-16) break;
  }
  for (int k = 0; k < 4; ++k)
    for (int it = 0; it < 2; ++it) {
      const C dk = dp(z[k]);
      if (dk != 0.0) z[k] -= p(z[k]) / dk;
    }
}

// Separate caustics of the binary lens (mass fractions and positions of sec. 4.1):
// critical points at nphi phases (m1 (z - x2)^2 + m2 (z - x1)^2 = e^{-i phi}
// (z - x1)^2 (z - x2)^2, i.e. |sum m_k/(conj z - x_k)^2| = 1), each joined to the
// nearest critical point of the next phase; each connected set is one critical
// curve, whose Eq. 2 image is one caustic.  Output rows (cx, cy, half_w, half_h,
// size) of the caustics' bounding boxes (size = the larger half-side), ordered by
// (round(1e9 cy), cx).
void caustic_components(double s, double q, int32_t nphi, std::vector<double>& out) {
  typedef std::complex<double> C;
  const double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  const double x1 = -s * q / (1.0 + q), x2 = s / (1.0 + q);
  const double S = x1 + x2, P = x1 * x2;
  std::vector<C> z((size_t)nphi * 4);
  C r[4];
  for (int p = 0; p < nphi; ++p) {
    const double ph = 2.0 * M_PI * p / nphi;
    const C e = std::polar(1.0, -ph);
    const C c[5] = {m1 * x2 * x2 + m2 * x1 * x1 - e * (P * P),
                    -2.0 * (m1 * x2 + m2 * x1) + 2.0 * e * (S * P),
                    (m1 + m2) - e * (S * S + 2.0 * P), 2.0 * e * S, -e};
    quartic_roots(c, r, p > 0);
    for (int k = 0; k < 4; ++k) z[(size_t)p * 4 + k] = r[k];
  }
  std::vector<int> parent((size_t)nphi * 4);
  for (size_t i = 0; i < parent.size(); ++i) parent[i] = (int)i;
  auto find = [&](int a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  };
  for (int p = 0; p < nphi; ++p) {
    const int pn = (p + 1) % nphi;
    for (int k = 0; k < 4; ++k) {
      int best = 0;
      double bd = std::abs(z[(size_t)pn * 4] - z[(size_t)p * 4 + k]);
      for (int j = 1; j < 4; ++j) {
        const double d = std::abs(z[(size_t)pn * 4 + j] - z[(size_t)p * 4 + k]);
        if (d < bd) {
          bd = d;
          best = j;
        }
      }
      const int a = find(p * 4 + k), b = find(pn * 4 + best);
      if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
  }
  struct Box {
    double x0, x1, y0, y1;
  };
  std::map<int, Box> boxes;
  for (size_t i = 0; i < z.size(); ++i) {
    const C zi = z[i];
    const C zeta = zi - m1 / std::conj(zi - x1) - m2 / std::conj(zi - x2);
    const int root = find((int)i);
    auto it = boxes.find(root);
    if (it == boxes.end()) {
      boxes[root] = {zeta.real(), zeta.real(), zeta.imag(), zeta.imag()};
    } else {
      Box& b = it->second;
      b.x0 = std::min(b.x0, zeta.real());
      b.x1 = std::max(b.x1, zeta.real());
      b.y0 = std::min(b.y0, zeta.imag());
      b.y1 = std::max(b.y1, zeta.imag());
    }
  }
  std::vector<std::array<double, 5>> rows;
  for (const auto& kv : boxes) {
    const Box& b = kv.second;
    const double hw = 0.5 * (b.x1 - b.x0), hh = 0.5 * (b.y1 - b.y0);
    rows.push_back({0.5 * (b.x0 + b.x1), 0.5 * (b.y0 + b.y1), hw, hh, std::max(hw, hh)});
  }
  std::sort(rows.begin(), rows.end(), [](const std::array<double, 5>& a, const std::array<double, 5>& b) {
    const long long ya = std::llround(a[1] * 1e9), yb = std::llround(b[1] * 1e9);
    return ya != yb ? ya < yb : a[0] < b[0];
  });
  out.clear();
  for (const auto& r5 : rows) out.insert(out.end(), r5.begin(), r5.end());
}
}  // namespace

// =============================================================================
extern "C" {

int morse_abi_version(void) { return MORSE_ABI_VERSION; }

const char* morse_last_error(const morse_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_thread_error.c_str();
}

int morse_ctx_create(int device, void* stream, morse_ctx** out) {
  if (!out) return fail(nullptr, MORSE_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(nullptr, MORSE_EINVAL, "no HIP device %d", device);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, MORSE_EHIP, "hipSetDevice failed");
  morse_ctx* c = new morse_ctx();
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return fail(nullptr, MORSE_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (hipStreamCreate(&c->capture_stream) != hipSuccess) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(nullptr, MORSE_EHIP, "hipStreamCreate failed");
  }
  *out = c;
  return MORSE_OK;
}

int morse_ctx_destroy(morse_ctx* ctx) {
  if (!ctx) return MORSE_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->refine_gexec) (void)hipGraphExecDestroy(ctx->refine_gexec);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->aux) (void)hipFree(ctx->aux);
  if (ctx->taps) (void)hipFree(ctx->taps);
  if (ctx->smeta.p) (void)hipFree(ctx->smeta.p);
  if (ctx->cmeta.p) (void)hipFree(ctx->cmeta.p);
  for (MetaBuf* mb : {&ctx->stack_taps, &ctx->fft_tw, &ctx->fft_spec, &ctx->lmeta})
    if (mb->p) (void)hipFree(mb->p);
  for (const auto& t : ctx->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MORSE_OK;
}

int morse_ctx_set_stream(morse_ctx* ctx, void* stream) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if ((hipStream_t)stream == ctx->stream) return MORSE_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  ctx->own_stream = false;
  ctx->stream = (hipStream_t)stream;
  return MORSE_OK;
}

int morse_ctx_synchronize(morse_ctx* ctx) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MORSE_OK;
}

int morse_ctx_set_timing(morse_ctx* ctx, uint32_t kernel_mask) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (kernel_mask >> 3) return fail(ctx, MORSE_EINVAL, "unknown kernel bits in mask 0x%x", kernel_mask);
  ctx->timing_mask = kernel_mask;
  return MORSE_OK;
}

int morse_ctx_kernel_time(morse_ctx* ctx, int32_t kernel, double* h_total_ms,
                          int64_t* h_launches, int32_t reset) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (kernel < 0 || kernel > 2) return fail(ctx, MORSE_EINVAL, "unknown kernel family %d", kernel);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, resolve_timers(ctx));
  if (h_total_ms) *h_total_ms = ctx->time_ms[kernel];
  if (h_launches) *h_launches = ctx->launches[kernel];
  if (reset) {
    ctx->time_ms[kernel] = 0.0;
    ctx->launches[kernel] = 0;
  }
  return MORSE_OK;
}

// ---------------------------------------------------------------------------
int morse_rayshoot(morse_ctx* ctx, double s, double q, const morse_grid2d* rays,
                   const morse_grid2d* window, int32_t row_begin, int32_t row_end,
                   uint32_t* d_counts, int32_t accumulate, uint64_t* d_stats) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check_lens(ctx, s, q))) return rc;
  if (!grid_ok(rays)) return fail(ctx, MORSE_EINVAL, "rays: invalid grid");
  if ((rc = check_window(ctx, window, "window"))) return rc;
  if (!d_counts) return fail(ctx, MORSE_EINVAL, "d_counts is NULL");
  if (row_begin < 0 || row_end > rays->ny || row_begin > row_end)
    return fail(ctx, MORSE_EINVAL, "row range [%d, %d) outside [0, %d]", row_begin, row_end, rays->ny);
  if ((double)rays->nx * (double)(row_end - row_begin) >= 4294967296.0)
    return fail(ctx, MORSE_ERANGE, "more than 2^32 - 1 rays in one call");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  RayParams p;
  p.m1 = (float)m1;
  p.m2 = (float)m2;
  p.x1 = (float)(-s * q / (1.0 + q));
  p.x2 = (float)(s / (1.0 + q));
  p.cx = (float)rays->cx;
  p.cy = (float)rays->cy;
  p.hx = (float)(rays->wx / rays->nx);
  p.hy = (float)(rays->wy / rays->ny);
  p.sx = (float)window->cx;
  p.sy = (float)window->cy;
  p.kx = (float)((double)window->nx / window->wx);
  p.ky = (float)((double)window->ny / window->wy);
  p.nx = rays->nx;
  p.ny = rays->ny;
  p.mx = window->nx;
  p.my = window->ny;
  p.row0 = row_begin;
  p.row1 = row_end;
  if (!accumulate) HIP_TRY(ctx, launch_fill_u32(d_counts, (size_t)window->nx * window->ny, 0u, ctx->stream));
  LaunchTimer tm{ctx, MORSE_KERNEL_RAYSHOOT};
  HIP_TRY(ctx, tm.begin(ctx->stream));
  HIP_TRY(ctx, launch_rayshoot(p, d_counts, (unsigned long long*)d_stats, ctx->stream));
  HIP_TRY(ctx, tm.end(ctx->stream));
  return MORSE_OK;
}

int morse_normalize_convolve(morse_ctx* ctx, const uint32_t* d_counts, const morse_grid2d* rays,
                             const morse_grid2d* window, double rho, float* d_map) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if (!grid_ok(rays)) return fail(ctx, MORSE_EINVAL, "rays: invalid grid");
  if ((rc = check_window(ctx, window, "window"))) return rc;
  if (!(std::isfinite(rho) && rho >= 0.0)) return fail(ctx, MORSE_EINVAL, "rho must be finite and >= 0");
  if (!d_counts || !d_map) return fail(ctx, MORSE_EINVAL, "d_counts / d_map is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double dx = window->wx / window->nx, dy = window->wy / window->ny;
  const double hx = (double)(float)(rays->wx / rays->nx), hy = (double)(float)(rays->wy / rays->ny);
  const float scale = (float)(hx * hy / (dx * dy));
  // the taps stay resident between calls with the same (rho, dx, dy): no host work,
  // upload or synchronisation in the steady state
  Hasher key;
  key.pod(rho);
  key.pod(dx);
  key.pod(dy);
  if (!ctx->taps || ctx->taps_key != key.h) {
    std::vector<float> w;
    std::vector<int32_t> off;
    if ((rc = disk_taps(ctx, rho, dx, dy, w, off))) return rc;
    const size_t w_bytes = (w.size() * sizeof(float) + 255) & ~size_t(255);
    const size_t need = w_bytes + off.size() * sizeof(int32_t);
    if (need > ctx->taps_size) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      if (ctx->taps) (void)hipFree(ctx->taps);
      ctx->taps = nullptr;
      ctx->taps_size = 0;
      if (hipMalloc((void**)&ctx->taps, need) != hipSuccess) {
        ctx->taps = nullptr;
        return fail(ctx, MORSE_ENOMEM, "taps allocation of %zu bytes failed", need);
      }
      ctx->taps_size = need;
    }
    ctx->taps_key = 0;
    if ((rc = upload(ctx, ctx->taps, w.data(), w.size() * sizeof(float)))) return rc;
    if ((rc = upload(ctx, ctx->taps + w_bytes, off.data(), off.size() * sizeof(int32_t)))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // host vectors go out of scope
    ctx->taps_key = key.h;
    ctx->taps_n = (int32_t)w.size();
    ctx->taps_wbytes = w_bytes;
  }
  const float* d_w = (const float*)ctx->taps;
  const int32_t* d_off = (const int32_t*)(ctx->taps + ctx->taps_wbytes);
  HIP_TRY(ctx, launch_normalize_convolve(d_counts, d_map, window->nx, window->ny, d_w, d_off,
                                         ctx->taps_n, scale, nullptr, ctx->stream));
  return MORSE_OK;
}

int morse_profile_weights(double rho, double dx, double dy, double gamma, double* h_w,
                          int64_t capacity, int32_t* h_rx, int32_t* h_ry) {
  if (!(std::isfinite(rho) && rho >= 0.0)) return fail(nullptr, MORSE_EINVAL, "rho must be finite and >= 0");
  if (!(std::isfinite(dx) && dx > 0.0 && std::isfinite(dy) && dy > 0.0))
    return fail(nullptr, MORSE_EINVAL, "pixel sizes must be finite and > 0");
  if (!(gamma >= 0.0 && gamma <= 1.0)) return fail(nullptr, MORSE_EINVAL, "gamma must lie in [0, 1]");
  if (!h_rx || !h_ry) return fail(nullptr, MORSE_EINVAL, "h_rx / h_ry is NULL");
  if (rho / std::min(dx, dy) > 4096.0) return fail(nullptr, MORSE_ERANGE, "rho spans more than 4096 pixels");
  int Rx = stencil_half(rho, dx), Ry = stencil_half(rho, dy);
  std::vector<double> q(1, 1.0);
  if (rho > 0.0) profile_quadrant(rho, dx, dy, gamma, Rx, Ry, q);
  // trim all-zero outer rings
  auto qw = [&](int a, int b) { return q[(size_t)b * (Rx + 1) + a]; };
  int tx = 0, ty = 0;
  for (int b = 0; b <= Ry; ++b)
    for (int a = 0; a <= Rx; ++a)
      if (qw(a, b) != 0.0) {
        tx = std::max(tx, a);
        ty = std::max(ty, b);
      }
  *h_rx = tx;
  *h_ry = ty;
  if (!h_w) return MORSE_OK;
  const int64_t need = (int64_t)(2 * tx + 1) * (2 * ty + 1);
  if (capacity < need)
    return fail(nullptr, MORSE_ERANGE, "capacity %lld < %lld weights", (long long)capacity, (long long)need);
  for (int b = -ty; b <= ty; ++b)
    for (int a = -tx; a <= tx; ++a) h_w[(int64_t)(b + ty) * (2 * tx + 1) + (a + tx)] = qw(std::abs(a), std::abs(b));
  return MORSE_OK;
}

int morse_convolve_stack(morse_ctx* ctx, const uint32_t* d_counts, const morse_grid2d* rays,
                         const morse_grid2d* window, const double* h_rho, int32_t n_rho,
                         double gamma, int32_t fft_min_taps, float* d_maps) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if (!grid_ok(rays)) return fail(ctx, MORSE_EINVAL, "rays: invalid grid");
  if ((rc = check_window(ctx, window, "window"))) return rc;
  if (n_rho < 0) return fail(ctx, MORSE_EINVAL, "n_rho < 0");
  if (n_rho == 0) return MORSE_OK;
  if (!h_rho || !d_counts || !d_maps) return fail(ctx, MORSE_EINVAL, "h_rho / d_counts / d_maps is NULL");
  if (!(gamma >= 0.0 && gamma <= 1.0)) return fail(ctx, MORSE_EINVAL, "gamma must lie in [0, 1]");
  for (int k = 0; k < n_rho; ++k)
    if (!(std::isfinite(h_rho[k]) && h_rho[k] >= 0.0))
      return fail(ctx, MORSE_EINVAL, "rho[%d] must be finite and >= 0", k);
  for (int k = 0; k < n_rho; ++k)
    if (h_rho[k] / std::min(window->wx / window->nx, window->wy / window->ny) > 4096.0)
      return fail(ctx, MORSE_ERANGE, "rho[%d] spans more than 4096 pixels", k);
  if (fft_min_taps <= 0) fft_min_taps = MORSE_STACK_FFT_MIN_TAPS;
  const int mx = window->nx, my = window->ny;
  const double dx = window->wx / mx, dy = window->wy / my;
  const double hx = (double)(float)(rays->wx / rays->nx), hy = (double)(float)(rays->wy / rays->ny);
  const size_t npx = (size_t)mx * my;
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  // Direct or FFT per radius; the direct taps of the whole call in one device table.
  // Both are kept in the context for the next call with the same arguments.
  Hasher skey;
  skey.pod(dx);
  skey.pod(dy);
  skey.pod(gamma);
  skey.pod(fft_min_taps);
  for (int k = 0; k < n_rho; ++k) skey.pod(h_rho[k]);
  auto& sp = ctx->stack_split;
  if (sp.key != skey.h || !ctx->stack_taps.p) {
    sp.key = 0;
    sp.direct_k.clear();
    sp.fft_k.clear();
    sp.ntaps.clear();
    sp.rmx = sp.rmy = 0;
    std::vector<float> w32;
    std::vector<int32_t> off;
    for (int k = 0; k < n_rho; ++k) {
      const int Rx = stencil_half(h_rho[k], dx), Ry = stencil_half(h_rho[k], dy);
      std::vector<float> wk;
      std::vector<int32_t> ok;
      bool direct = Rx <= 15 && Ry <= 15;
      if (direct) {
        if ((rc = profile_taps(ctx, h_rho[k], dx, dy, gamma, wk, ok))) return rc;
        direct = (int64_t)wk.size() < (int64_t)fft_min_taps || wk.size() == 1;
      }
      if (direct) {
        sp.direct_k.push_back(k);
        sp.ntaps.push_back((int32_t)wk.size());
        w32.insert(w32.end(), wk.begin(), wk.end());
        off.insert(off.end(), ok.begin(), ok.end());
      } else {
        sp.fft_k.push_back(k);
        sp.rmx = std::max(sp.rmx, Rx);
        sp.rmy = std::max(sp.rmy, Ry);
      }
    }
    const size_t w_bytes = (w32.size() * sizeof(float) + 255) & ~size_t(255);
    if ((rc = reserve_meta(ctx, ctx->stack_taps, std::max<size_t>(256, w_bytes + off.size() * sizeof(int32_t)))))
      return rc;
    if ((rc = upload(ctx, ctx->stack_taps.p, w32.data(), w32.size() * sizeof(float)))) return rc;
    if ((rc = upload(ctx, ctx->stack_taps.p + w_bytes, off.data(), off.size() * sizeof(int32_t)))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the host tables go out of scope
    sp.w_bytes = w_bytes;
    sp.key = skey.h;
  }
  const std::vector<int>& direct_k = sp.direct_k;
  const std::vector<int>& fft_k = sp.fft_k;
  // FFT sizes checked before any launch
  auto pow2_at_least = [](int64_t v) {
    int64_t n = 2;
    while (n < v) n <<= 1;
    return n;
  };
  const int64_t nx64 = pow2_at_least((int64_t)mx + 2 * sp.rmx), ny64 = pow2_at_least((int64_t)my + 2 * sp.rmy);
  if (!fft_k.empty() && (nx64 > kFftMaxN || ny64 > kFftMaxN))
    return fail(ctx, MORSE_ERANGE, "FFT convolution needs %lld x %lld > %d per side (map plus twice the stencil radius)",
                (long long)nx64, (long long)ny64, kFftMaxN);
  {
    const float scale = (float)(hx * hy / (dx * dy));
    const size_t w_bytes = sp.w_bytes;
    size_t at = 0;
    for (size_t u = 0; u < direct_k.size(); ++u) {
      const float* d_w = (const float*)(ctx->stack_taps.p) + at;
      const int32_t* d_off = (const int32_t*)(ctx->stack_taps.p + w_bytes) + 2 * at;
      HIP_TRY(ctx, launch_normalize_convolve(d_counts, d_maps + (size_t)direct_k[u] * npx, mx, my, d_w,
                                             d_off, sp.ntaps[u], scale, nullptr, ctx->stream));
      at += (size_t)sp.ntaps[u];
    }
  }
  if (fft_k.empty()) return MORSE_OK;

  // FFT path: twiddles, profile-pair transforms (kept in the context), then one
  // forward transform of the counts and one inverse transform per pair.
  FftGrid g;
  g.nx = (int32_t)nx64;
  g.ny = (int32_t)ny64;
  {
    Hasher key;
    key.pod(g.nx);
    key.pod(g.ny);
    const size_t need = (size_t)(g.nx + g.ny) * sizeof(double2);
    if (ctx->fft_tw.key != key.h || ctx->fft_tw.size < need) {
      if ((rc = reserve_meta(ctx, ctx->fft_tw, need))) return rc;
      ctx->fft_tw.key = 0;
      std::vector<double2> t((size_t)g.nx + g.ny);
      for (int m = 0; m < g.nx; ++m) {
        const double th = 2.0 * M_PI * m / g.nx;
        t[m] = make_double2(std::cos(th), -std::sin(th));
      }
      for (int m = 0; m < g.ny; ++m) {
        const double th = 2.0 * M_PI * m / g.ny;
        t[(size_t)g.nx + m] = make_double2(std::cos(th), -std::sin(th));
      }
      if ((rc = upload(ctx, ctx->fft_tw.p, t.data(), need))) return rc;
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      ctx->fft_tw.key = key.h;
    }
    g.tw_x = (const double2*)ctx->fft_tw.p;
    g.tw_y = (const double2*)ctx->fft_tw.p + g.nx;
  }
  const size_t nf = (size_t)g.nx * g.ny;
  const size_t fbytes = nf * sizeof(double2);
  const int pairs = (int)(fft_k.size() + 1) / 2;
  Plan pl;
  const size_t i0 = pl.add(fbytes), i1 = pl.add(fbytes), i2 = pl.add(fbytes);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  double2* B[3] = {(double2*)pl.ptr(ctx, i0), (double2*)pl.ptr(ctx, i1), (double2*)pl.ptr(ctx, i2)};
  {
    Hasher key;
    key.pod(g.nx);
    key.pod(g.ny);
    key.pod(dx);
    key.pod(dy);
    key.pod(gamma);
    for (int k : fft_k) key.pod(h_rho[k]);
    const size_t need = (size_t)pairs * fbytes;
    if (ctx->fft_spec.key != key.h || ctx->fft_spec.size < need) {
      if ((rc = reserve_meta(ctx, ctx->fft_spec, need))) return rc;
      ctx->fft_spec.key = 0;
      for (int p = 0; p < pairs; ++p) {
        std::vector<double> q[2];
        int rx[2] = {0, 0}, ry[2] = {0, 0};
        const int nk = (2 * p + 1 < (int)fft_k.size()) ? 2 : 1;
        for (int u = 0; u < nk; ++u) {
          const double rho = h_rho[fft_k[2 * p + u]];
          rx[u] = stencil_half(rho, dx);
          ry[u] = stencil_half(rho, dy);
          profile_quadrant(rho, dx, dy, gamma, rx[u], ry[u], q[u]);
        }
        // the quadrant tables go through B[2] (free until the counts transform)
        double* dq0 = (double*)B[2];
        double* dq1 = dq0 + q[0].size();
        if ((q[0].size() + q[1].size()) * sizeof(double) > fbytes)
          return fail(ctx, MORSE_ERANGE, "profile tables exceed the transform buffer");
        if ((rc = upload(ctx, dq0, q[0].data(), q[0].size() * sizeof(double)))) return rc;
        if (nk == 2 && (rc = upload(ctx, dq1, q[1].data(), q[1].size() * sizeof(double)))) return rc;
        HIP_TRY(ctx, launch_fft_rows_taps(g, dq0, rx[0], ry[0], nk == 2 ? dq1 : nullptr, rx[1], ry[1],
                                          B[0], ctx->stream));
        double2* spec = (double2*)ctx->fft_spec.p + (size_t)p * nf;
        double2* res = nullptr;
        const ColTransform full{-1, g.nx, g.nx, g.nx, 0, 0, nullptr, g.ny};
        HIP_TRY(ctx, launch_fft_cols(g, full, B[0], spec, B[1], &res, ctx->stream));
        if (res != spec) HIP_TRY(ctx, hipMemcpyAsync(spec, res, fbytes, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // q goes out of scope
      }
      ctx->fft_spec.key = key.h;
    }
  }
  // counts: half spectrum [ny][nx/2 + 1] (the padded image is real)
  const int32_t h = g.nx / 2 + 1;
  double2* X = nullptr;
  HIP_TRY(ctx, launch_fft_rows_counts(g, d_counts, mx, my, B[0], ctx->stream));
  const ColTransform fwd{-1, h, h, h, my, 0, nullptr, g.ny};
  HIP_TRY(ctx, launch_fft_cols(g, fwd, B[0], B[1], B[2], &X, ctx->stream));
  double2* other = (X == B[1]) ? B[2] : B[1];
  const double scale = hx * hy / (dx * dy) / ((double)g.nx * (double)g.ny);
  for (int p = 0; p < pairs; ++p) {
    const double2* spec = (const double2*)ctx->fft_spec.p + (size_t)p * nf;
    double2* Y = nullptr;
    const ColTransform inv{1, g.nx, h, g.nx, 0, h, spec, my};
    HIP_TRY(ctx, launch_fft_cols(g, inv, X, B[0], other, &Y, ctx->stream));
    float* m1 = d_maps + (size_t)fft_k[2 * p] * npx;
    float* m2 = (2 * p + 1 < (int)fft_k.size()) ? d_maps + (size_t)fft_k[2 * p + 1] * npx : nullptr;
    HIP_TRY(ctx, launch_fft_rows_store(g, Y, mx, my, scale, m1, m2, ctx->stream));
  }
  return MORSE_OK;
}

// ---------------------------------------------------------------------------
// Caustic-centred lines (sec. 4.2) and the minimum-magnification filter (sec. 4.3).

int morse_caustics(double s, double q, int32_t nphi, double* h_out, int32_t capacity,
                   int32_t* h_n) {
  if (!(std::isfinite(s) && s > 0.0)) return fail(nullptr, MORSE_EINVAL, "s must be finite and > 0");
  if (!(q > 0.0 && q <= 1.0)) return fail(nullptr, MORSE_EINVAL, "q must lie in (0, 1]");
  if (nphi < 16 || nphi > (1 << 20)) return fail(nullptr, MORSE_EINVAL, "nphi must lie in [16, 2^20]");
  if (!h_n) return fail(nullptr, MORSE_EINVAL, "h_n is NULL");
  std::vector<double> c;
  caustic_components(s, q, nphi, c);
  const int32_t n = (int32_t)(c.size() / 5);
  *h_n = n;
  if (h_out) {
    if (capacity < n) return fail(nullptr, MORSE_ERANGE, "capacity %d < %d caustics", capacity, n);
    std::copy(c.begin(), c.end(), h_out);
  }
  return MORSE_OK;
}

int morse_caustic_lines(const double* h_caustics, int32_t n_caustics, const double* h_r, int32_t n_r,
                        const double* h_phi, int32_t n_phi, double* h_lines) {
  if (n_caustics < 0 || n_r < 0 || n_phi < 0) return fail(nullptr, MORSE_EINVAL, "negative count");
  if ((n_caustics && !h_caustics) || (n_r && !h_r) || (n_phi && !h_phi) ||
      (!h_lines && n_caustics && n_r && n_phi))
    return fail(nullptr, MORSE_EINVAL, "NULL array");
  int64_t o = 0;
  for (int k = 0; k < n_caustics; ++k) {
    const double cx = h_caustics[5 * k], cy = h_caustics[5 * k + 1], size = h_caustics[5 * k + 4];
    for (int j = 0; j < n_r; ++j)
      for (int l = 0; l < n_phi; ++l) {
        const double ph = h_phi[l], sn = std::sin(ph), cn = std::cos(ph);
        h_lines[3 * o] = h_r[j] * size - cx * sn + cy * cn;
        h_lines[3 * o + 1] = ph;
        h_lines[3 * o + 2] = cx * cn + cy * sn;
        ++o;
      }
  }
  return MORSE_OK;
}

int morse_line_filter(morse_ctx* ctx, const morse_map_view* map, const double* d_lines, int64_t n,
                      double a_min, float* d_best, uint8_t* d_keep, int64_t* d_kept,
                      int64_t* d_count, int64_t* h_count) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if (!map || !map->d_map) return fail(ctx, MORSE_EINVAL, "map is NULL");
  if ((rc = check_window(ctx, &map->window, "map window"))) return rc;
  if ((rc = check_quad_size(ctx, map, 1))) return rc;
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if (!std::isfinite(a_min)) return fail(ctx, MORSE_EINVAL, "a_min must be finite");
  if (n > 0 && (!d_lines || !d_best || !d_keep)) return fail(ctx, MORSE_EINVAL, "d_lines / d_best / d_keep is NULL");
  if (n == 0) {
    if (d_count) HIP_TRY(ctx, launch_fill_u64((uint64_t*)d_count, 1, 0ull, ctx->stream));
    if (h_count) *h_count = 0;
    return MORSE_OK;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const morse_grid2d& w = map->window;
  const double R = 0.5 * std::sqrt(w.wx * w.wx + w.wy * w.wy);
  const double kmax = std::max(w.nx / w.wx, w.ny / w.wy);
  const double ns64 = std::ceil(2.0 * R * kmax) + 1.0;
  if (ns64 > 1.0e7) return fail(ctx, MORSE_ERANGE, "more than 1e7 samples per line");
  const bool compact = d_kept || d_count || h_count;
  Plan pl;
  const size_t iq = pl.add(quad_bytes(w.nx, w.ny));
  const size_t is = pl.add(compact ? compact_scratch_elems(n) * sizeof(int64_t) : 0);
  const size_t ic = pl.add(sizeof(int64_t));
  if ((rc = reserve(ctx, pl.total()))) return rc;
  std::vector<MapC> hm(1, make_mapc(map->d_map, w));
  assign_quads(hm, pl.ptr(ctx, iq));
  if ((rc = reserve_meta(ctx, ctx->lmeta, sizeof(MapC)))) return rc;
  Hasher key;
  key.pod(ctx->lmeta.p);
  key.bytes(hm.data(), sizeof(MapC));
  if (ctx->lmeta.key != key.h) {
    ctx->lmeta.key = 0;
    if ((rc = upload(ctx, ctx->lmeta.p, hm.data(), sizeof(MapC)))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // hm goes out of scope
    ctx->lmeta.key = key.h;
  }
  HIP_TRY(ctx, launch_quad_pack((const MapC*)ctx->lmeta.p, hm.data(), 1, ctx->stream));
  LineFilterArgs a;
  a.m = hm[0];
  a.lines = d_lines;
  a.n = n;
  a.cxw = w.cx;
  a.cyw = w.cy;
  a.half_diag = R;
  a.ns = (int32_t)ns64;
  a.h = (float)(2.0 * R / (ns64 - 1.0));
  a.amin = (float)a_min;
  a.best = d_best;
  a.keep = d_keep;
  HIP_TRY(ctx, launch_line_filter(a, ctx->stream));
  if (compact) {
    int64_t* cnt = d_count ? d_count : (int64_t*)pl.ptr(ctx, ic);
    HIP_TRY(ctx, launch_compact(d_keep, n, (int64_t*)pl.ptr(ctx, is), d_kept, cnt, ctx->stream));
    if (h_count) {
      HIP_TRY(ctx, hipMemcpyAsync(h_count, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
  }
  return MORSE_OK;
}

int morse_lines_to_trajectories(morse_ctx* ctx, const double* d_lines, const int64_t* d_kept,
                                int64_t n_kept, const double* h_t0, int32_t n_t0, const double* h_tE,
                                int32_t n_tE, double* d_params) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (n_kept < 0 || n_t0 < 0 || n_tE < 0) return fail(ctx, MORSE_EINVAL, "negative count");
  const int64_t total = n_kept * (int64_t)n_t0 * n_tE;
  if (total == 0) return MORSE_OK;
  if (!d_lines || !h_t0 || !h_tE || !d_params) return fail(ctx, MORSE_EINVAL, "NULL array");
  for (int32_t b = 0; b < n_tE; ++b)
    if (!(std::isfinite(h_tE[b]) && h_tE[b] > 0.0)) return fail(ctx, MORSE_EINVAL, "tE[%d] must be finite and > 0", b);
  int rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Plan pl;
  const size_t i0 = pl.add(sizeof(double) * n_t0), i1 = pl.add(sizeof(double) * n_tE);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  double* t0 = (double*)pl.ptr(ctx, i0);
  double* tE = (double*)pl.ptr(ctx, i1);
  if ((rc = upload(ctx, t0, h_t0, sizeof(double) * n_t0))) return rc;
  if ((rc = upload(ctx, tE, h_tE, sizeof(double) * n_tE))) return rc;
  HIP_TRY(ctx, launch_lines_to_traj(d_lines, d_kept, n_kept, t0, n_t0, tE, n_tE, d_params, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the host axes are read during the call only
  return MORSE_OK;
}

int morse_build_map(morse_ctx* ctx, double s, double q, const morse_grid2d* rays,
                    const morse_grid2d* window, double rho, uint32_t* d_counts, float* d_map,
                    morse_map_stats* h_stats) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check_lens(ctx, s, q))) return rc;
  if (!grid_ok(rays)) return fail(ctx, MORSE_EINVAL, "rays: invalid grid");
  if ((rc = check_window(ctx, window, "window"))) return rc;
  if (!(std::isfinite(rho) && rho >= 0.0)) return fail(ctx, MORSE_EINVAL, "rho must be finite and >= 0");
  if (!d_map) return fail(ctx, MORSE_EINVAL, "d_map is NULL");
  if ((double)rays->nx * (double)rays->ny >= 4294967296.0)
    return fail(ctx, MORSE_ERANGE, "more than 2^32 - 1 rays");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double dx = window->wx / window->nx, dy = window->wy / window->ny;
  std::vector<float> w;
  std::vector<int32_t> off;
  if ((rc = disk_taps(ctx, rho, dx, dy, w, off))) return rc;
  const size_t npx = (size_t)window->nx * window->ny;
  Plan pl;
  const size_t ic = pl.add(d_counts ? 0 : npx * 4), is = pl.add(3 * 8 + 8),
               iw = pl.add(w.size() * 4), io = pl.add(off.size() * 4);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  uint32_t* counts = d_counts ? d_counts : (uint32_t*)pl.ptr(ctx, ic);
  uint64_t* stats = (uint64_t*)pl.ptr(ctx, is);
  uint32_t* maxc = (uint32_t*)(stats + 3);
  float* d_w = (float*)pl.ptr(ctx, iw);
  int32_t* d_off = (int32_t*)pl.ptr(ctx, io);
  if ((rc = upload(ctx, d_w, w.data(), w.size() * 4))) return rc;
  if ((rc = upload(ctx, d_off, off.data(), off.size() * 4))) return rc;
  HIP_TRY(ctx, launch_fill_u64(stats, 4, 0ull, ctx->stream));
  if ((rc = morse_rayshoot(ctx, s, q, rays, window, 0, rays->ny, counts, 0, stats))) return rc;
  const double hx = (double)(float)(rays->wx / rays->nx), hy = (double)(float)(rays->wy / rays->ny);
  const float scale = (float)(hx * hy / (dx * dy));
  HIP_TRY(ctx, launch_normalize_convolve(counts, d_map, window->nx, window->ny, d_w, d_off,
                                         (int32_t)w.size(), scale, maxc, ctx->stream));
  // the small host vectors must outlive their (possibly staged) copies
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (h_stats) {
    uint64_t hs[4];
    HIP_TRY(ctx, hipMemcpy(hs, stats, sizeof(hs), hipMemcpyDeviceToHost));
    h_stats->rays_total = (uint64_t)rays->nx * (uint64_t)rays->ny;
    h_stats->rays_out = hs[0];
    h_stats->rays_nonfinite = hs[1];
    h_stats->rays_zero_axis = hs[2];
    h_stats->rays_in = h_stats->rays_total - hs[0] - hs[1];
    h_stats->max_count = (uint32_t)(hs[3] & 0xffffffffu);
    h_stats->reserved = 0;
    if (h_stats->max_count > (1u << 24))
      return fail(ctx, MORSE_ERANGE, "a pixel holds %u > 2^24 rays (FP32 normalisation inexact)",
                  h_stats->max_count);
  }
  return MORSE_OK;
}

}  // extern "C"

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
};

int validate_search(morse_ctx* ctx, const morse_map_view* maps, int32_t n_maps,
                    const morse_lightcurves* lcs, const morse_trajectories* trajs) {
  int rc;
  if (!maps || n_maps <= 0) return fail(ctx, MORSE_EINVAL, "need n_maps >= 1 maps");
  for (int i = 0; i < n_maps; ++i) {
    if (!maps[i].d_map) return fail(ctx, MORSE_EINVAL, "map %d: d_map is NULL", i);
    if ((rc = check_window(ctx, &maps[i].window, "map window"))) return rc;
  }
  if (!lcs || lcs->n_events <= 0 || !lcs->h_offsets || !lcs->h_t_ref || !lcs->d_t || !lcs->d_flux ||
      !lcs->d_weight)
    return fail(ctx, MORSE_EINVAL, "light curves: missing arrays or n_events <= 0");
  if (lcs->h_offsets[0] != 0) return fail(ctx, MORSE_EINVAL, "light curves: offsets[0] must be 0");
  for (int e = 0; e < lcs->n_events; ++e) {
    const int64_t n = lcs->h_offsets[e + 1] - lcs->h_offsets[e];
    if (n < 3) return fail(ctx, MORSE_EINVAL, "event %d has %lld < 3 points", e, (long long)n);
    if (n > (1ll << 30)) return fail(ctx, MORSE_ERANGE, "event %d too long", e);
    if (!std::isfinite(lcs->h_t_ref[e])) return fail(ctx, MORSE_EINVAL, "event %d: t_ref not finite", e);
  }
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
  Plan pl;
  const size_t i_quad = pl.add(quad_region_bytes(maps, n_maps)),
               i_sums = pl.add(24 * (size_t)sp.n_events), i_cnt = pl.add(4 * kQueueWords),
               i_wF = pl.add(8 * (size_t)sp.n_pts), i_tc = pl.add(sizeof(TrajC) * (size_t)n_tc),
               i_chi = pl.add(need_chi2 ? 8 * (size_t)n_out : 0),
               i_tk = pl.add(k > 0 ? topk_scratch_bytes(sp.n_events, k) : 0);
  if ((rc = reserve(ctx, pl.total()))) return rc;
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
  return launch_traj_prep_list(trajs->d_params, n, sp.tc, st);
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

// ---------------------------------------------------------------------------
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
  if (!lcs || lcs->n_events <= 0 || !lcs->h_offsets || !lcs->h_t_ref || !lcs->d_t || !lcs->d_flux ||
      !lcs->d_weight)
    return fail(ctx, MORSE_EINVAL, "light curves: missing arrays or n_events <= 0");
  for (int e = 0; e < lcs->n_events; ++e)
    if (lcs->h_offsets[e + 1] - lcs->h_offsets[e] < 3)
      return fail(ctx, MORSE_EINVAL, "event %d has fewer than 3 points", e);
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
  const size_t i_tc = pl.add(sizeof(TrajC) * (size_t)n), i_tE = pl.add(8 * (size_t)n);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  GradArgs a{};
  a.tc = (TrajC*)pl.ptr(ctx, i_tc);
  a.tEv = (double*)pl.ptr(ctx, i_tE);
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
  HIP_TRY(ctx, launch_cand_prep(a, ctx->stream));
  LaunchTimer tm{ctx, MORSE_KERNEL_GRADIENT};
  HIP_TRY(ctx, tm.begin(ctx->stream));
  HIP_TRY(ctx, launch_chi2_grad(a, ctx->stream));
  HIP_TRY(ctx, tm.end(ctx->stream));
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
               i_tE = pl.add(8 * (size_t)n);
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
  // The rounds are captured once per argument set and replayed: start (anchor copy,
  // state reset, first-trial constants), steps + 1 rounds of (evaluation, update with
  // the next trial's constants), write-back.
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
  // start, steps + 1 rounds, write-back; with `timing`, events bracket each evaluation
  auto enqueue = [&](hipStream_t cs, bool timing) -> hipError_t {
    hipError_t e = launch_refine_init(s, a, d_params, anchor, cs);
    for (int r = 0; r <= opts->steps && e == hipSuccess; ++r) {
      LaunchTimer tm{ctx, MORSE_KERNEL_GRADIENT};
      if (timing) e = tm.begin(cs);
      if (e == hipSuccess) e = launch_chi2_grad(a, cs);
      if (e == hipSuccess && timing) e = tm.end(cs);
      if (e == hipSuccess)
        e = launch_lbfgs_update(s, a, r, ft, gt, r == 0 ? d_chi2_init : nullptr, cs);
    }
    if (e == hipSuccess) e = launch_lbfgs_finish(s, d_params, d_chi2_out, cs);
    return e;
  };
  if (timed(ctx, MORSE_KERNEL_GRADIENT)) {  // same kernels, launched one by one
    HIP_TRY(ctx, enqueue(ctx->stream, true));
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
    hipError_t e = enqueue(cs, false);
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
