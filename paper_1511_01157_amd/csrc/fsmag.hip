// Finite-source magnification by image-centred ray shooting on gfx950 (sec. 5 of
// McDougall & Albrow 2015: point source beyond 10 rho from the caustic, otherwise polar
// grids grown around the source's images and integrated with the source profile).
//
// Classification, one wavefront per source: the distance from the source centre to the
// nearest caustic point; far sources take the point-source magnification of their
// images (Eqs. 3-4, one thread each), near ones are listed.  Regions, one 256-lane
// workgroup per listed source: every lane solves the lens equation for one of the
// centre and n_b boundary points (the quintic of Eq. 2, FP64 Aberth-Ehrlich), the
// images and the critical points whose caustic image lies inside the source become
// seeds in polar coordinates about the centre of mass; the seeds are sorted in LDS
// (bitonic), cut into angular runs at gaps wider than `gap` and each run at radial
// gaps; every region grows until none of its sides maps inside the source (side samples
// spread over the lanes); overlapping regions merge.  Integration, one 512-lane
// workgroup per (source, region): column by column (one lane per theta column, radial
// segments with the limb crossing linear in f = rho^2 - |zeta - zeta_s|^2 and the
// square-root edge of the limb-darkened profile integrated exactly), then the region
// cut to its inside cells and integrated again; a last kernel adds each source's region
// integrals in region order.  All arithmetic is FP64.

#include "fsmag.h"

namespace morse {

namespace {

constexpr int kFsThreads = 256;
constexpr int kSeedCap = 2048;   // seeds per source (a power of two for the sort)
constexpr int kRegionCap = kFsRegionCap;
constexpr int kCritSeeds = 512;  // critical-point seeds at most

__global__ void k_fill_u32_fs(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0u;
}

struct cd {
  double x, y;
};
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ double cabs(cd a) { return hypot(a.x, a.y); }
// a / b: directly as a conj(b) / |b|^2 while |b|^2 stays well inside the FP64 range,
// else scaled (Smith).
__device__ __forceinline__ cd cdivc(cd a, cd b) {
  const double n = b.x * b.x + b.y * b.y;
  if (n > 1e-280 && n < 1e280) {
    const double s = 1.0 / n;
    return {(a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s};
  }
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return {(a.x + a.y * r) / d, (a.y - a.x * r) / d};
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return {(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}
__device__ __forceinline__ cd crecip(cd b) { return cdivc(cd{1.0, 0.0}, b); }

struct Lens {
  double m1, m2, x1, x2;
};

// Eq. 2: zeta = z - m1/(conj z - x1) - m2/(conj z - x2).
__device__ __forceinline__ cd lens_eq(const Lens& L, cd z) {
  const cd w1 = {z.x - L.x1, -z.y}, w2 = {z.x - L.x2, -z.y};
  return csub(csub(z, cscale(crecip(w1), L.m1)), cscale(crecip(w2), L.m2));
}

// |zeta(z) - zs|^2 by Eq. 2 with each lens term written as m_k (z - x_k) / |z - x_k|^2,
// the conjugate's reciprocal: one division per lens and no square root (the samples of
// the image-centred integration and the growth test; a sample on a lens gives inf or
// NaN, which compare as outside the source).
__device__ __forceinline__ double lens_dist2(const Lens& L, cd z, cd zs) {
  const double d1 = z.x - L.x1, d2 = z.x - L.x2, yy = z.y * z.y;
  const double a1 = L.m1 / (d1 * d1 + yy), a2 = L.m2 / (d2 * d2 + yy);
  const double ex = ((z.x - a1 * d1) - a2 * d2) - zs.x;
  const double ey = ((z.y - a1 * z.y) - a2 * z.y) - zs.y;
  return ex * ex + ey * ey;
}

// The quintic whose roots contain the images of zeta.  With Q = (z - x1)(z - x2) and
// P_k = (conj zeta - x_k) Q + m1 (z - x2) + m2 (z - x1) (so 1/(conj z - x_k) = Q/P_k on
// an image, from the conjugate of Eq. 2), Eq. 2 times P1 P2 reads
//   (z - zeta) P1 P2 - Q (m1 P2 + m2 P1) = 0.
// Coefficients ascending, a[0..5].
__device__ void quintic(const Lens& L, cd zeta, cd (&a)[6]) {
  const cd zb = {zeta.x, -zeta.y};
  const double q0 = L.x1 * L.x2, q1 = -(L.x1 + L.x2);  // Q = q0 + q1 z + z^2
  const double lin0 = -(L.m1 * L.x2 + L.m2 * L.x1), lin1 = L.m1 + L.m2;
  cd P1[3], P2[3];
  const cd c1 = {zb.x - L.x1, zb.y}, c2 = {zb.x - L.x2, zb.y};
  P1[0] = cadd(cscale(c1, q0), cd{lin0, 0.0});
  P1[1] = cadd(cscale(c1, q1), cd{lin1, 0.0});
  P1[2] = c1;
  P2[0] = cadd(cscale(c2, q0), cd{lin0, 0.0});
  P2[1] = cadd(cscale(c2, q1), cd{lin1, 0.0});
  P2[2] = c2;
  cd T[5] = {};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[i + j] = cadd(T[i + j], cmul(P1[i], P2[j]));
  cd U[3];
  for (int i = 0; i < 3; ++i) U[i] = cadd(cscale(P2[i], L.m1), cscale(P1[i], L.m2));
  const double Q[3] = {q0, q1, 1.0};
  cd QU[5] = {};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) QU[i + j] = cadd(QU[i + j], cscale(U[j], Q[i]));
  // (z - zeta) T
  a[0] = csub(cmul(cd{-zeta.x, -zeta.y}, T[0]), QU[0]);
  for (int k = 1; k < 5; ++k) a[k] = csub(csub(T[k - 1], cmul(zeta, T[k])), QU[k]);
  a[5] = T[4];
}

__device__ __forceinline__ void poly_eval(const cd (&a)[6], cd z, cd& p, cd& dp) {
  p = a[5];
  dp = {0.0, 0.0};
  for (int k = 4; k >= 0; --k) {
    dp = cadd(cmul(dp, z), p);
    p = cadd(cmul(p, z), a[k]);
  }
}

// Roots of the quintic: Aberth-Ehrlich from a circle (Cauchy bound) until the largest
// relative step is below 1e-14 or, below 1e-9, stops halving (the rounding floor of
// the polynomial's evaluation, which ill-conditioned roots never get under), then two
// Newton steps per root.
__device__ void quintic_roots(const cd (&a)[6], cd (&z)[5]) {
  const cd inv5 = crecip(a[5]);
  double rad = 0.0;
  for (int i = 0; i < 5; ++i) rad = fmax(rad, cabs(cmul(a[i], inv5)));
  rad = 1.0 + rad;
  for (int k = 0; k < 5; ++k) {
    double sn, cs;
    sincos(0.4 + 2.0 * M_PI * k / 5.0, &sn, &cs);
    z[k] = {rad * cs, rad * sn};
  }
  double prev = __builtin_inf();
  for (int it = 0; it < 200; ++it) {
    double moved = 0.0;
    for (int k = 0; k < 5; ++k) {
      cd p, dp;
      poly_eval(a, z[k], p, dp);
      if (p.x == 0.0 && p.y == 0.0) continue;
      const cd ratio = cdivc(p, dp);
      cd rep = {0.0, 0.0};
      for (int j = 0; j < 5; ++j)
        if (j != k) rep = cadd(rep, crecip(csub(z[k], z[j])));
      const cd step = cdivc(ratio, csub(cd{1.0, 0.0}, cmul(ratio, rep)));
      if (!(isfinite(step.x) && isfinite(step.y))) continue;
      z[k] = csub(z[k], step);
      moved = fmax(moved, cabs(step) / (1.0 + cabs(z[k])));
    }
    if (moved < 1e-14 || (moved < 1e-9 && moved >= 0.5 * prev)) break;
    prev = moved;
  }
  for (int k = 0; k < 5; ++k)
    for (int it = 0; it < 2; ++it) {
      cd p, dp;
      poly_eval(a, z[k], p, dp);
      if (dp.x != 0.0 || dp.y != 0.0) z[k] = csub(z[k], cdivc(p, dp));
    }
}

// Images of zeta: the 5 roots when all satisfy Eq. 2 to 1e-6 (1 + |zeta|), else the 3
// with the smallest residuals (ties: the lower root index) when at least 3 do, else
// those that do.  sel[k] marks the images among the roots z[k]; returns their number.
// Written without indexing by a runtime value, so the arrays stay in registers.
__device__ __forceinline__ int images_of(const Lens& L, cd zeta, cd (&z)[5], bool (&sel)[5]) {
  cd a[6];
  quintic(L, zeta, a);
  quintic_roots(a, z);
  double res[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double r = cabs(csub(lens_eq(L, z[k]), zeta));
    res[k] = isfinite(r) ? r : __builtin_inf();
  }
  const double tol = 1e-6 * (1.0 + cabs(zeta));
  int nvalid = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) nvalid += res[k] < tol ? 1 : 0;
  const int nimg = nvalid >= 5 ? 5 : (nvalid >= 3 ? 3 : nvalid);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int rank = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) rank += (res[j] < res[k] || (res[j] == res[k] && j < k)) ? 1 : 0;
    sel[k] = rank < nimg;
  }
  return nimg;
}

__device__ double point_source_A(const Lens& L, cd zeta) {
  cd z[5];
  bool sel[5];
  images_of(L, zeta, z, sel);
  double A = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const cd w1 = {z[k].x - L.x1, -z[k].y}, w2 = {z[k].x - L.x2, -z[k].y};
    const cd g = cadd(cscale(crecip(cmul(w1, w1)), L.m1), cscale(crecip(cmul(w2, w2)), L.m2));
    const double ag = cabs(g);
    A += sel[k] ? fabs(1.0 / (1.0 - ag * ag)) : 0.0;
  }
  return A;
}

// One wavefront per source: the lanes share the caustic points and a butterfly minimum
// gives the distance.  Far sources are marked for the point-source kernel, near ones
// listed for the image-centred kernel.
__global__ __launch_bounds__(256) void k_fs_classify(FsArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < a.n;
       i += waves) {
    const cd zs = {a.zeta[2 * i], a.zeta[2 * i + 1]};
    double dmin = __builtin_inf();
    for (int32_t j = lane; j < a.n_crit; j += kWave) {
      const double d = cabs(csub(cd{a.caus[2 * j], a.caus[2 * j + 1]}, zs));
      if (d < dmin) dmin = d;  // NaN points (a massless companion) never win
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dmin = fmin(dmin, __shfl_xor(dmin, off));
    if (lane == 0) {
      if (dmin > a.near * a.rho) {
        a.nreg[i] = -1;
      } else {
        a.nreg[i] = 0;
        const uint32_t slot = atomicAdd(a.near_count, 1u);
        a.near_list[slot] = (int32_t)i;
      }
    }
  }
}

// Point-source magnification of the sources marked far (one thread per source).
__global__ __launch_bounds__(256) void k_fs_point(FsArgs a) {
  const Lens L{a.m1, a.m2, a.x1, a.x2};
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.n || a.nreg[i] != -1) return;
  a.A[i] = point_source_A(L, cd{a.zeta[2 * i], a.zeta[2 * i + 1]});
}

// ---------------------------------------------------------------------------------
// Image-centred kernel.
struct Region {
  double r0, r1, t0, t1;
};

__device__ __forceinline__ bool is_ring(const Region& g) { return g.t1 - g.t0 >= 2.0 * M_PI; }

// Ascending bitonic sort of n = kSeedCap keys with a payload (all lanes).
__device__ void bitonic(double* key, double* v1, double* v2) {
  for (int k = 2; k <= kSeedCap; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kSeedCap; i += kFsThreads) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          if ((key[i] > key[l]) == up) {
            double t = key[i];
            key[i] = key[l];
            key[l] = t;
            t = v1[i];
            v1[i] = v1[l];
            v1[l] = t;
            t = v2[i];
            v2[i] = v2[l];
            v2[l] = t;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ bool inside_source(const Lens& L, cd z, cd zs, double rho) {
  return lens_dist2(L, z, zs) < rho * rho;
}

// numpy.linspace(a, b, n)[k]
__device__ __forceinline__ double linspace_at(double a, double b, int n, int k) {
  return k == n - 1 ? b : a + k * ((b - a) / (n - 1));
}

__device__ __forceinline__ bool theta_overlap(const Region& a, const Region& b) {
  if (is_ring(a) || is_ring(b)) return true;
  const double k = rint(((a.t0 + a.t1) - (b.t0 + b.t1)) / (4.0 * M_PI));
  const double b0 = b.t0 + 2.0 * M_PI * k, b1 = b.t1 + 2.0 * M_PI * k;
  return !(b1 < a.t0 || b0 > a.t1);
}

__device__ Region region_union(const Region& a, const Region& b) {
  Region u{fmin(a.r0, b.r0), fmax(a.r1, b.r1), -M_PI, M_PI};
  if (is_ring(a) || is_ring(b)) return u;
  const double k = rint(((a.t0 + a.t1) - (b.t0 + b.t1)) / (4.0 * M_PI));
  u.t0 = fmin(a.t0, b.t0 + 2.0 * M_PI * k);
  u.t1 = fmax(a.t1, b.t1 + 2.0 * M_PI * k);
  if (u.t1 - u.t0 >= 2.0 * M_PI) {
    u.t0 = -M_PI;
    u.t1 = M_PI;
  }
  return u;
}

struct Shared {
  double key[kSeedCap], r[kSeedCap], th[kSeedCap];
  int run[kSeedCap];
  Region reg[kRegionCap];
  int ired[4][kFsThreads];
  int n_seed, n_reg, flag[4];
};

// Integral of the profile over one region and the bounds of its inside nodes (all
// NT lanes of the workgroup; box = {k0, k1, j0, j1}, k1 < 0 when nothing is inside).
template <int NT>
struct IntShared {
  double red[NT];
  int ired[4][NT];
};

template <int NT>
__device__ double integrate_region(const FsArgs& a, const Lens& L, cd zs, const Region& g,
                                   IntShared<NT>& sh, int (&box)[4]) {
  const double rho2 = a.rho * a.rho;
  const double dth = (g.t1 - g.t0) / a.n_theta;
  const double dr = (g.r1 - g.r0) / a.n_r;
  const double c_ld = 1.5 * a.gamma / a.rho;
  double acc = 0.0;
  int k0 = 1 << 30, k1 = -1, j0 = 1 << 30, j1 = -1;
  for (int j = threadIdx.x; j < a.n_theta; j += NT) {
    double sn, cs;
    sincos(g.t0 + (j + 0.5) * dth, &sn, &cs);
    double col = 0.0, fa = 0.0, ra = 0.0;
    bool any = false;
    for (int k = 0; k <= a.n_r; ++k) {
      const double r = g.r0 + k * dr;
      const double f = rho2 - lens_dist2(L, cd{r * cs, r * sn}, zs);
      if (f > 0.0) {
        any = true;
        k0 = min(k0, k);
        k1 = max(k1, k);
      }
      if (k > 0 && (fa > 0.0 || f > 0.0)) {
        // the inside part [lo, hi] of the segment, the limb where f (linear) is zero
        const bool ina = fa > 0.0, inb = f > 0.0;
        const double rs = ra + dr * fa / (fa - f);
        const double lo = ina ? ra : rs, hi = inb ? ra + dr : rs;
        const double sa = ina ? sqrt(fa) : 0.0, sb = inb ? sqrt(f) : 0.0;
        const double ms = (sa + sb > 0.0) ? (2.0 / 3.0) * (sa * sa + sa * sb + sb * sb) / (sa + sb) : 0.0;
        const double len = hi - lo, rm = 0.5 * (lo + hi);
        col += (1.0 - a.gamma) * rm * len + c_ld * rm * len * ms;
      }
      fa = f;
      ra = r;
    }
    acc += col;
    if (any) {
      j0 = min(j0, j);
      j1 = max(j1, j);
    }
  }
  sh.red[threadIdx.x] = acc;
  sh.ired[0][threadIdx.x] = k0;
  sh.ired[1][threadIdx.x] = k1;
  sh.ired[2][threadIdx.x] = j0;
  sh.ired[3][threadIdx.x] = j1;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {  // fixed tree: the same sum every time
    if ((int)threadIdx.x < w) {
      sh.red[threadIdx.x] += sh.red[threadIdx.x + w];
      sh.ired[0][threadIdx.x] = min(sh.ired[0][threadIdx.x], sh.ired[0][threadIdx.x + w]);
      sh.ired[1][threadIdx.x] = max(sh.ired[1][threadIdx.x], sh.ired[1][threadIdx.x + w]);
      sh.ired[2][threadIdx.x] = min(sh.ired[2][threadIdx.x], sh.ired[2][threadIdx.x + w]);
      sh.ired[3][threadIdx.x] = max(sh.ired[3][threadIdx.x], sh.ired[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  const double total = sh.red[0] * dth;
  for (int q = 0; q < 4; ++q) box[q] = sh.ired[q][0];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kFsThreads) void k_fs_regions(FsArgs a) {
  __shared__ Shared sh;
  const Lens L{a.m1, a.m2, a.x1, a.x2};
  const int tid = threadIdx.x;
  const double two_pi = 2.0 * M_PI;
  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const int64_t i = a.near_list[a.item0 + item];
    const cd zs = {a.zeta[2 * i], a.zeta[2 * i + 1]};
    if (tid == 0) sh.n_seed = 0;
    __syncthreads();
    // seeds: images of the centre (j = 0) and of the boundary points, then the
    // critical points whose caustic image lies inside the source
    for (int j = tid; j <= a.n_b; j += kFsThreads) {
      cd p = zs;
      if (j > 0) {
        double sn, cs;
        sincos(two_pi * ((j - 1) + 0.5) / a.n_b, &sn, &cs);
        p = {zs.x + a.rho * cs, zs.y + a.rho * sn};
      }
      cd z[5];
      bool sel[5];
      images_of(L, p, z, sel);
#pragma unroll
      for (int k = 0; k < 5; ++k)
        if (sel[k]) {
          const int slot = atomicAdd(&sh.n_seed, 1);
          if (slot < kSeedCap) {
            sh.r[slot] = cabs(z[k]);
            sh.th[slot] = atan2(z[k].y, z[k].x);
          }
        }
    }
    // at most kCritSeeds of them: those of every m-th phase, m the smallest stride
    // >= ceil(count / kCritSeeds) that keeps at most kCritSeeds
    int m = 1;
    for (int pass = 0;; ++pass) {
      int c = 0;
      for (int32_t j = tid; j < a.n_crit; j += kFsThreads)
        c += (((j >> 2) % m) == 0 && cabs(csub(cd{a.caus[2 * j], a.caus[2 * j + 1]}, zs)) < a.rho) ? 1 : 0;
      sh.ired[0][tid] = c;
      __syncthreads();
      for (int w = kFsThreads / 2; w > 0; w >>= 1) {
        if (tid < w) sh.ired[0][tid] += sh.ired[0][tid + w];
        __syncthreads();
      }
      const int count = sh.ired[0][0];
      __syncthreads();
      if (count <= kCritSeeds) break;
      m = pass == 0 ? (count + kCritSeeds - 1) / kCritSeeds : m + 1;
    }
    for (int32_t j = tid; j < a.n_crit; j += kFsThreads) {
      const cd c = {a.caus[2 * j], a.caus[2 * j + 1]};
      if (((j >> 2) % m) == 0 && cabs(csub(c, zs)) < a.rho) {
        const int slot = atomicAdd(&sh.n_seed, 1);
        if (slot < kSeedCap) {
          const cd z = {a.crit[2 * j], a.crit[2 * j + 1]};
          sh.r[slot] = cabs(z);
          sh.th[slot] = atan2(z.y, z.x);
        }
      }
    }
    __syncthreads();
    const int ns = sh.n_seed;
    if (ns > kSeedCap || ns == 0) {  // uniform
      if (tid == 0) {
        a.A[i] = __builtin_nan("");
        a.nreg[i] = -2;
        a.reg_count[item] = 0;
      }
      __syncthreads();
      continue;
    }
    // 1. seeds by angle
    for (int j = tid; j < kSeedCap; j += kFsThreads) sh.key[j] = j < ns ? sh.th[j] : __builtin_inf();
    __syncthreads();
    bitonic(sh.key, sh.r, sh.th);
    // 2. angular runs: cuts at gaps wider than `gap` (circularly); walking from the
    // seed after the first cut, run ids and angles unwrapped from each run's first seed
    if (tid == 0) {
      int first = -1;
      for (int j = 0; j < ns; ++j) {
        const double nxt = j + 1 < ns ? sh.th[j + 1] : sh.th[0] + two_pi;
        sh.run[j] = (nxt - sh.th[j] > a.gap) ? 1 : 0;  // cut after seed j
        if (first < 0 && sh.run[j]) first = j;
      }
      sh.flag[0] = first < 0 ? 1 : 0;
      if (first < 0) {  // no cut: one ring
        double r0 = sh.r[0], r1 = sh.r[0];
        for (int j = 1; j < ns; ++j) {
          r0 = fmin(r0, sh.r[j]);
          r1 = fmax(r1, sh.r[j]);
        }
        sh.reg[0] = Region{r0, r1, -M_PI, M_PI};
        sh.n_reg = 1;
      } else {
        int run = 0;
        bool fresh = true;
        double start = 0.0;
        for (int m = 0; m < ns; ++m) {
          const int j = (first + 1 + m) % ns;
          const int cut = sh.run[j];
          if (fresh) start = sh.th[j];
          fresh = false;
          if (sh.th[j] < start) sh.th[j] += two_pi;
          sh.run[j] = run;
          sh.key[j] = run * 1.0e6 + sh.r[j];  // radii stay far below 1e6
          if (cut) {
            ++run;
            fresh = true;
          }
        }
      }
    }
    __syncthreads();
    if (!sh.flag[0]) {
      // 3. seeds by (run, r); parts of a run split where the radius jumps
      bitonic(sh.key, sh.r, sh.th);
      if (tid == 0) {
        int nr = 0;
        for (int j = 0; j < ns; ++j) {
          const int run = (int)floor(sh.key[j] / 1.0e6);
          const bool fresh = j == 0 || run != (int)floor(sh.key[j - 1] / 1.0e6) ||
                             sh.r[j] - sh.r[j - 1] > fmax(a.gap * sh.r[j], 4.0 * a.rho);
          if (fresh) {
            if (nr == kRegionCap) {
              nr = kRegionCap + 1;
              break;
            }
            sh.reg[nr++] = Region{sh.r[j], sh.r[j], sh.th[j], sh.th[j]};
          } else {
            Region& g = sh.reg[nr - 1];
            g.r1 = sh.r[j];
            g.t0 = fmin(g.t0, sh.th[j]);
            g.t1 = fmax(g.t1, sh.th[j]);
          }
        }
        sh.n_reg = nr;
      }
      __syncthreads();
    }
    if (sh.n_reg > kRegionCap) {  // uniform
      if (tid == 0) {
        a.A[i] = __builtin_nan("");
        a.nreg[i] = -3;
        a.reg_count[item] = 0;
      }
      __syncthreads();
      continue;
    }
    // 4. padding: 10 % of the extent plus rho in r and rho / r1 in theta
    if (tid == 0) {
      for (int g = 0; g < sh.n_reg; ++g) {
        Region& R = sh.reg[g];
        const double dr = 0.1 * (R.r1 - R.r0) + a.rho;
        R.r0 = fmax(0.0, R.r0 - dr);
        R.r1 = R.r1 + dr;
        if (R.t1 - R.t0 < two_pi) {
          const double dt = 0.1 * (R.t1 - R.t0) + a.rho / fmax(R.r1, 1e-12);
          R.t0 -= dt;
          R.t1 += dt;
        }
        if (R.t1 - R.t0 >= two_pi) {
          R.t0 = -M_PI;
          R.t1 = M_PI;
        }
      }
    }
    __syncthreads();
    // 5. growth: a side with a sample inside the source moves out by a quarter extent
    for (int g = 0; g < sh.n_reg; ++g) {
      for (int it = 0; it < a.n_grow; ++it) {
        if (tid < 4) sh.flag[tid] = 0;
        __syncthreads();
        const Region R = sh.reg[g];
        const int sides = is_ring(R) ? 2 : 4;
        for (int t = tid; t < sides * a.n_side; t += kFsThreads) {
          const int side = t / a.n_side, k = t % a.n_side;
          double rr, tt;
          if (side < 2) {
            rr = side == 0 ? R.r0 : R.r1;
            tt = linspace_at(R.t0, R.t1, a.n_side, k);
          } else {
            rr = linspace_at(R.r0, R.r1, a.n_side, k);
            tt = side == 2 ? R.t0 : R.t1;
          }
          double sn, cs;
          sincos(tt, &sn, &cs);
          if (inside_source(L, cd{rr * cs, rr * sn}, zs, a.rho)) sh.flag[side] = 1;
        }
        __syncthreads();
        const int h0 = sh.flag[0], h1 = sh.flag[1], h2 = sh.flag[2], h3 = sh.flag[3];
        __syncthreads();
        if (!(h0 | h1 | h2 | h3)) break;
        if (tid == 0) {
          Region& W = sh.reg[g];
          const double dr = 0.25 * (W.r1 - W.r0), dt = 0.25 * (W.t1 - W.t0);
          if (h0) W.r0 = fmax(0.0, W.r0 - dr);
          if (h1) W.r1 = W.r1 + dr;
          if (h2) W.t0 = W.t0 - dt;
          if (h3) W.t1 = W.t1 + dt;
          if (W.t1 - W.t0 >= two_pi) {
            W.t0 = -M_PI;
            W.t1 = M_PI;
          }
        }
        __syncthreads();
      }
    }
    // 6. overlapping regions merge (first overlapping pair first, until none overlap)
    if (tid == 0) {
      bool changed = true;
      while (changed) {
        changed = false;
        for (int p = 0; p < sh.n_reg && !changed; ++p)
          for (int q = p + 1; q < sh.n_reg && !changed; ++q) {
            const Region& A = sh.reg[p];
            const Region& B = sh.reg[q];
            if (!(B.r1 < A.r0 || B.r0 > A.r1) && theta_overlap(A, B)) {
              sh.reg[p] = region_union(A, B);
              for (int m = q; m + 1 < sh.n_reg; ++m) sh.reg[m] = sh.reg[m + 1];
              --sh.n_reg;
              changed = true;
            }
          }
      }
    }
    __syncthreads();
    // 7. the regions and their work items for the integration kernel
    const int n_reg = sh.n_reg;
    if (tid < n_reg) {
      const Region R = sh.reg[tid];
      double* out = a.regs + 4 * (item * kFsRegionCap + tid);
      out[0] = R.r0;
      out[1] = R.r1;
      out[2] = R.t0;
      out[3] = R.t1;
    }
    if (tid == 0) {
      a.reg_count[item] = n_reg;
      sh.flag[0] = (int)atomicAdd(a.work_count, (uint32_t)n_reg);
    }
    __syncthreads();
    if (tid < n_reg) a.work[sh.flag[0] + tid] = (uint32_t)(item * kFsRegionCap + tid);
    __syncthreads();
  }
}

// 8. One workgroup per (source, region): the region's integral, then up to n_shrink
// times the region cut to its inside cells (plus one cell) and integrated again.
constexpr int kIntThreads = 512;
__global__ __launch_bounds__(kIntThreads) void k_fs_integrate(FsArgs a) {
  __shared__ IntShared<kIntThreads> sh;
  const Lens L{a.m1, a.m2, a.x1, a.x2};
  const uint32_t n_work = *a.work_count;
  for (uint32_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const uint32_t slot = a.work[w];
    const int64_t i = a.near_list[a.item0 + slot / kFsRegionCap];
    const cd zs = {a.zeta[2 * i], a.zeta[2 * i + 1]};
    const double* rg = a.regs + 4 * (int64_t)slot;
    Region R{rg[0], rg[1], rg[2], rg[3]};
    int box[4];
    double val = integrate_region<kIntThreads>(a, L, zs, R, sh, box);
    for (int it = 0; it < a.n_shrink; ++it) {
      if (box[1] < 0) break;
      const double dr = (R.r1 - R.r0) / a.n_r;
      const int n0 = max(box[0] - 1, 0), n1 = min(box[1] + 1, a.n_r);
      Region N = {R.r0 + n0 * dr, R.r0 + n1 * dr, R.t0, R.t1};
      if (!is_ring(R)) {
        const double dth = (R.t1 - R.t0) / a.n_theta;
        N.t0 = R.t0 + max(box[2] - 1, 0) * dth;
        N.t1 = R.t0 + min(box[3] + 2, a.n_theta) * dth;
      }
      if (N.r0 == R.r0 && N.r1 == R.r1 && N.t0 == R.t0 && N.t1 == R.t1) break;
      R = N;
      val = integrate_region<kIntThreads>(a, L, zs, R, sh, box);
    }
    if (threadIdx.x == 0) a.reg_val[slot] = val;
  }
}

// 9. Per source: the region integrals summed in region order (one thread per source).
__global__ __launch_bounds__(256) void k_fs_finish(FsArgs a) {
  const int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (item >= a.n_items) return;
  const int32_t nr = a.reg_count[item];
  if (nr <= 0) return;  // a seed or region failure, already written
  const int64_t i = a.near_list[a.item0 + item];
  double total = 0.0;
  for (int g = 0; g < nr; ++g) total += a.reg_val[item * kFsRegionCap + g];
  a.A[i] = total / (M_PI * a.rho * a.rho);
  a.nreg[i] = nr;
}

// Source positions along a trajectory (FP64): tau = (t - t0)/tE,
// zeta = tau (cos a, sin a) + u0 (-sin a, cos a).
__global__ __launch_bounds__(256) void k_traj_positions(const double* t, int64_t n, double t0,
                                                        double u0, double tE, double ca, double sa,
                                                        double* zeta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double tau = (t[i] - t0) / tE;
    zeta[2 * i] = tau * ca - u0 * sa;
    zeta[2 * i + 1] = tau * sa + u0 * ca;
  }
}

}  // namespace

hipError_t launch_traj_positions(const double* t, int64_t n, double t0, double u0, double tE,
                                 double alpha, double* zeta, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_traj_positions, dim3((unsigned)blocks), dim3(256), 0, st, t, n, t0, u0, tE,
                     cos(alpha), sin(alpha), zeta);
  return hipGetLastError();
}

hipError_t launch_fs_classify(const FsArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32_fs, dim3(1), dim3(64), 0, st, a.near_count);
  int64_t blocks = (a.n + 3) / 4;  // four sources (wavefronts) per workgroup
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fs_classify, dim3((unsigned)blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_fs_point, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fs_images(const FsArgs& a, int32_t max_blocks, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.n_b < 1 || a.n_side < 2 || a.n_r < 1 || a.n_theta < 1 || a.n_grow < 0 || a.n_shrink < 0 ||
      a.n_items > kFsBatch)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_u32_fs, dim3(1), dim3(64), 0, st, a.work_count);
  const int64_t blocks = a.n_items < max_blocks ? a.n_items : max_blocks;
  hipLaunchKernelGGL(k_fs_regions, dim3((unsigned)blocks), dim3(kFsThreads), 0, st, a);
  hipLaunchKernelGGL(k_fs_integrate, dim3((unsigned)max_blocks), dim3(kIntThreads), 0, st, a);
  hipLaunchKernelGGL(k_fs_finish, dim3((unsigned)((a.n_items + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace morse
