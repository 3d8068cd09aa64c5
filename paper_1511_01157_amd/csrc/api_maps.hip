// C ABI, map build: ray shooting, normalisation and convolution with source profiles
// (uniform and limb-darkened disks, one radius or a stack of radii), and the host
// preparations they need (exact disk/pixel overlap weights, binary32 constants).

#include "host.h"

using namespace morse;
using namespace morse::host;

namespace {

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


}  // namespace

extern "C" {

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
    tap_reach(off, ctx->taps_rx, ctx->taps_ry);
  }
  const float* d_w = (const float*)ctx->taps;
  const int32_t* d_off = (const int32_t*)(ctx->taps + ctx->taps_wbytes);
  HIP_TRY(ctx, launch_normalize_convolve(d_counts, d_map, window->nx, window->ny, d_w, d_off,
                                         ctx->taps_n, ctx->taps_rx, ctx->taps_ry, scale, nullptr,
                                         ctx->stream));
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
    sp.reach.clear();
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
        int32_t rx, ry;
        tap_reach(ok, rx, ry);
        sp.reach.push_back(rx);
        sp.reach.push_back(ry);
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
                                             d_off, sp.ntaps[u], sp.reach[2 * u], sp.reach[2 * u + 1],
                                             scale, nullptr, ctx->stream));
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
  int32_t rx, ry;
  tap_reach(off, rx, ry);
  HIP_TRY(ctx, launch_normalize_convolve(counts, d_map, window->nx, window->ny, d_w, d_off,
                                         (int32_t)w.size(), rx, ry, scale, maxc, ctx->stream));
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
