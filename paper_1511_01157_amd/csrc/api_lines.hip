// C ABI, caustic-centred trajectories: caustic geometry on the host (critical-curve
// quartic, separate caustics), lines at radial distances from the caustic centres, the
// minimum-magnification line filter and the expansion of kept lines into trajectories.

#include "host.h"

using namespace morse;
using namespace morse::host;

#include <complex>

namespace {

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
}  // namespace

namespace morse {
namespace host {
// Critical points at nphi equally spaced phases (4 per phase, phase-major).
void critical_points(double s, double q, int32_t nphi, std::vector<std::complex<double>>& z) {
  typedef std::complex<double> C;
  const double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  const double x1 = -s * q / (1.0 + q), x2 = s / (1.0 + q);
  const double S = x1 + x2, P = x1 * x2;
  z.assign((size_t)nphi * 4, C(0.0, 0.0));
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
}
}  // namespace host
}  // namespace morse

namespace {

void caustic_components(double s, double q, int32_t nphi, std::vector<double>& out) {
  typedef std::complex<double> C;
  const double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  const double x1 = -s * q / (1.0 + q), x2 = s / (1.0 + q);
  std::vector<C> z;
  critical_points(s, q, nphi, z);
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

namespace {

// Shared set-up of the line filter and the peak library: validation, the map packed
// into cells (descriptor resident in ctx->lmeta), the sampling of the lines across the
// window, and the workspace of the compaction.
int setup_lines(morse_ctx* ctx, const morse_map_view* map, const double* d_lines, int64_t n,
                double a_min, bool compact, LineFilterArgs& a, Plan& pl, size_t& is, size_t& ic) {
  int rc;
  if (!map || !map->d_map) return fail(ctx, MORSE_EINVAL, "map is NULL");
  if ((rc = check_window(ctx, &map->window, "map window"))) return rc;
  if ((rc = check_quad_size(ctx, map, 1))) return rc;
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if (!std::isfinite(a_min)) return fail(ctx, MORSE_EINVAL, "a_min must be finite");
  if (n == 0) return MORSE_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const morse_grid2d& w = map->window;
  const double R = 0.5 * std::sqrt(w.wx * w.wx + w.wy * w.wy);
  const double kmax = std::max(w.nx / w.wx, w.ny / w.wy);
  const double ns64 = std::ceil(2.0 * R * kmax) + 1.0;
  if (ns64 > 1.0e7) return fail(ctx, MORSE_ERANGE, "more than 1e7 samples per line");
  const size_t iq = pl.add(quad_bytes(w.nx, w.ny));
  is = pl.add(compact ? compact_scratch_elems(n) * sizeof(int64_t) : 0);
  ic = pl.add(sizeof(int64_t));
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
  a.m = hm[0];
  a.lines = d_lines;
  a.n = n;
  a.cxw = w.cx;
  a.cyw = w.cy;
  a.half_diag = R;
  a.ns = (int32_t)ns64;
  a.h = (float)(2.0 * R / (ns64 - 1.0));
  a.amin = (float)a_min;
  return MORSE_OK;
}

int finish_empty(morse_ctx* ctx, int64_t* d_count, int64_t* h_count) {
  if (d_count) HIP_TRY(ctx, launch_fill_u64((uint64_t*)d_count, 1, 0ull, ctx->stream));
  if (h_count) *h_count = 0;
  return MORSE_OK;
}

// Kept lines in ascending order (optional list, device and host counts).
int compact_kept(morse_ctx* ctx, const Plan& pl, size_t is, size_t ic, const uint8_t* d_keep,
                 int64_t n, int64_t* d_kept, int64_t* d_count, int64_t* h_count) {
  if (!(d_kept || d_count || h_count)) return MORSE_OK;
  int64_t* cnt = d_count ? d_count : (int64_t*)pl.ptr(ctx, ic);
  HIP_TRY(ctx, launch_compact(d_keep, n, (int64_t*)pl.ptr(ctx, is), d_kept, cnt, ctx->stream));
  if (h_count) {
    HIP_TRY(ctx, hipMemcpyAsync(h_count, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return MORSE_OK;
}

}  // namespace

extern "C" {

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
  if (n > 0 && (!d_lines || !d_best || !d_keep)) return fail(ctx, MORSE_EINVAL, "d_lines / d_best / d_keep is NULL");
  LineFilterArgs a;
  Plan pl;
  size_t is = 0, ic = 0;
  if ((rc = setup_lines(ctx, map, d_lines, n, a_min, d_kept || d_count || h_count, a, pl, is, ic)))
    return rc;
  if (n == 0) return finish_empty(ctx, d_count, h_count);
  a.best = d_best;
  a.keep = d_keep;
  HIP_TRY(ctx, launch_line_filter(a, ctx->stream));
  return compact_kept(ctx, pl, is, ic, d_keep, n, d_kept, d_count, h_count);
}

int morse_line_peaks(morse_ctx* ctx, const morse_map_view* map, const double* d_lines, int64_t n,
                     double a_min, int32_t min_peaks, double hysteresis, int32_t max_peaks,
                     float* d_best, int32_t* d_npeaks, float* d_peak_tau, float* d_peak_A,
                     uint8_t* d_keep, int64_t* d_kept, int64_t* d_count, int64_t* h_count) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if (!(std::isfinite(hysteresis) && hysteresis >= 0.0 && hysteresis < 1.0))
    return fail(ctx, MORSE_EINVAL, "hysteresis must lie in [0, 1)");
  if (max_peaks < 1 || max_peaks > 64) return fail(ctx, MORSE_EINVAL, "max_peaks must lie in [1, 64]");
  if (min_peaks < 0) return fail(ctx, MORSE_EINVAL, "min_peaks < 0");
  if (n > 0 && (!d_lines || !d_best || !d_npeaks || !d_peak_tau || !d_peak_A || !d_keep))
    return fail(ctx, MORSE_EINVAL, "NULL device array");
  LinePeakArgs a;
  Plan pl;
  size_t is = 0, ic = 0;
  if ((rc = setup_lines(ctx, map, d_lines, n, a_min, d_kept || d_count || h_count, a.f, pl, is, ic)))
    return rc;
  if (n == 0) return finish_empty(ctx, d_count, h_count);
  a.f.best = d_best;
  a.f.keep = d_keep;
  a.up = (float)(1.0 + hysteresis);
  a.down = (float)(1.0 - hysteresis);
  a.min_peaks = min_peaks;
  a.kmax = max_peaks;
  a.npeaks = d_npeaks;
  a.ptau = d_peak_tau;
  a.pA = d_peak_A;
  HIP_TRY(ctx, launch_line_peaks(a, ctx->stream));
  return compact_kept(ctx, pl, is, ic, d_keep, n, d_kept, d_count, h_count);
}

int morse_peak_starts(morse_ctx* ctx, const double* d_lines, const int64_t* d_kept, int64_t n,
                      const int32_t* d_npeaks, const float* d_peak_tau, const float* d_peak_A,
                      int32_t max_peaks, const double* h_tp, int32_t n_tp, double tE,
                      double* d_start) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if (n_tp != 1 && n_tp != 2) return fail(ctx, MORSE_EINVAL, "n_tp must be 1 or 2");
  if (max_peaks < 1 || max_peaks > 64) return fail(ctx, MORSE_EINVAL, "max_peaks must lie in [1, 64]");
  if (!h_tp || !std::isfinite(h_tp[0]) || (n_tp == 2 && !(std::isfinite(h_tp[1]) && h_tp[1] > h_tp[0])))
    return fail(ctx, MORSE_EINVAL, "peak times must be finite and increasing");
  if (n_tp == 1 && !(std::isfinite(tE) && tE > 0.0)) return fail(ctx, MORSE_EINVAL, "tE must be finite and > 0");
  if (n == 0) return MORSE_OK;
  if (!d_lines || !d_npeaks || !d_peak_tau || !d_peak_A || !d_start)
    return fail(ctx, MORSE_EINVAL, "NULL device array");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  PeakStartArgs a;
  a.lines = d_lines;
  a.kept = d_kept;
  a.n = n;
  a.npeaks = d_npeaks;
  a.ptau = d_peak_tau;
  a.pA = d_peak_A;
  a.kmax = max_peaks;
  a.n_tp = n_tp;
  a.tp1 = h_tp[0];
  a.tp2 = n_tp == 2 ? h_tp[1] : 0.0;
  a.tE = tE;
  a.start = d_start;
  HIP_TRY(ctx, launch_peak_starts(a, ctx->stream));
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

}  // extern "C"
