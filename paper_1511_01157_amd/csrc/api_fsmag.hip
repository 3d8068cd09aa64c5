// C ABI, finite-source magnification by image-centred ray shooting (sec. 5): the
// critical curves on the host, then the proximity kernel and the image-centred kernel.

#include "host.h"
#include "fsmag.h"

using namespace morse;
using namespace morse::host;

extern "C" {

int morse_fs_magnification(morse_ctx* ctx, double s, double q, const double* d_zeta, int64_t n,
                           double rho, double gamma, const morse_fs_opts* opts, double* d_A,
                           int32_t* d_nreg) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check_lens(ctx, s, q))) return rc;
  if (!(std::isfinite(rho) && rho > 0.0)) return fail(ctx, MORSE_EINVAL, "rho must be finite and > 0");
  if (!(gamma >= 0.0 && gamma <= 1.0)) return fail(ctx, MORSE_EINVAL, "gamma must lie in [0, 1]");
  if (!opts) return fail(ctx, MORSE_EINVAL, "opts is NULL");
  const morse_fs_opts& o = *opts;
  if (o.n_b < 8 || o.n_b > 1024 || o.n_crit < 16 || o.n_crit > (1 << 16) || o.n_side < 2 ||
      o.n_side > 4096 || o.n_grow < 0 || o.n_grow > 1000 || o.n_r < 2 || o.n_r > 65536 ||
      o.n_theta < 2 || o.n_theta > 65536 || o.n_shrink < 0 || o.n_shrink > 16)
    return fail(ctx, MORSE_EINVAL, "opts out of range");
  if (!(std::isfinite(o.near) && o.near >= 0.0 && std::isfinite(o.gap) && o.gap > 0.0))
    return fail(ctx, MORSE_EINVAL, "near must be >= 0 and gap > 0");
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if (n == 0) return MORSE_OK;
  if (!d_zeta || !d_A) return fail(ctx, MORSE_EINVAL, "d_zeta / d_A is NULL");
  if (n > (int64_t)1 << 31) return fail(ctx, MORSE_ERANGE, "more than 2^31 sources");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double m1 = 1.0 / (1.0 + q), m2 = q / (1.0 + q);
  const double x1 = -s * q / (1.0 + q), x2 = s / (1.0 + q);
  // critical points and their caustic images (Eq. 2), host FP64, resident in the context
  // until a call needs another (s, q, phases)
  const size_t nc = (size_t)o.n_crit * 4;
  if ((rc = reserve_meta(ctx, ctx->fs_crit, 32 * nc))) return rc;
  Hasher key;
  key.pod(ctx->fs_crit.p);
  key.pod(s);
  key.pod(q);
  key.pod(o.n_crit);
  if (ctx->fs_crit.key != key.h) {
    ctx->fs_crit.key = 0;
    std::vector<std::complex<double>> zc;
    critical_points(s, q, o.n_crit, zc);
    std::vector<double> buf(4 * nc);
    for (size_t j = 0; j < nc; ++j) {
      const std::complex<double> z = zc[j];
      const std::complex<double> zeta = z - m1 / std::conj(z - x1) - m2 / std::conj(z - x2);
      buf[2 * j] = z.real();
      buf[2 * j + 1] = z.imag();
      buf[2 * nc + 2 * j] = zeta.real();
      buf[2 * nc + 2 * j + 1] = zeta.imag();
    }
    if ((rc = upload(ctx, ctx->fs_crit.p, buf.data(), 32 * nc))) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // buf goes out of scope
    ctx->fs_crit.key = key.h;
  }
  Plan pl;
  const int64_t batch = std::min<int64_t>(n, kFsBatch);
  const size_t i_list = pl.add(4 * (size_t)n), i_cnt = pl.add(4),
               i_nreg = pl.add(d_nreg ? 0 : 4 * (size_t)n),
               i_regs = pl.add(32 * (size_t)batch * kFsRegionCap), i_rc = pl.add(4 * (size_t)batch),
               i_rv = pl.add(8 * (size_t)batch * kFsRegionCap),
               i_work = pl.add(4 * (size_t)batch * kFsRegionCap), i_wc = pl.add(4);
  if ((rc = reserve(ctx, pl.total()))) return rc;
  FsArgs a;
  a.m1 = m1;
  a.m2 = m2;
  a.x1 = x1;
  a.x2 = x2;
  a.zeta = d_zeta;
  a.n = n;
  a.rho = rho;
  a.gamma = gamma;
  a.crit = (const double*)ctx->fs_crit.p;
  a.caus = (const double*)ctx->fs_crit.p + 2 * nc;
  a.n_crit = (int32_t)nc;
  a.n_b = o.n_b;
  a.n_side = o.n_side;
  a.n_grow = o.n_grow;
  a.n_r = o.n_r;
  a.n_theta = o.n_theta;
  a.n_shrink = o.n_shrink;
  a.near = o.near;
  a.gap = o.gap;
  a.A = d_A;
  a.nreg = d_nreg ? d_nreg : (int32_t*)pl.ptr(ctx, i_nreg);
  a.near_list = (int32_t*)pl.ptr(ctx, i_list);
  a.near_count = (uint32_t*)pl.ptr(ctx, i_cnt);
  a.regs = (double*)pl.ptr(ctx, i_regs);
  a.reg_count = (int32_t*)pl.ptr(ctx, i_rc);
  a.reg_val = (double*)pl.ptr(ctx, i_rv);
  a.work = (uint32_t*)pl.ptr(ctx, i_work);
  a.work_count = (uint32_t*)pl.ptr(ctx, i_wc);
  HIP_TRY(ctx, launch_fs_classify(a, ctx->stream));
  // the number of sources near a caustic sizes the image-centred passes
  uint32_t n_near = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&n_near, a.near_count, 4, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t b0 = 0; b0 < (int64_t)n_near; b0 += kFsBatch) {
    a.item0 = b0;
    a.n_items = std::min<int64_t>(kFsBatch, (int64_t)n_near - b0);
    HIP_TRY(ctx, launch_fs_images(a, 4 * ctx->num_cu, ctx->stream));
  }
  return MORSE_OK;
}

int morse_trajectory_positions(morse_ctx* ctx, const double* h_params, const double* d_t, int64_t n,
                               double* d_zeta) {
  if (!ctx) return fail(nullptr, MORSE_EINVAL, "ctx is NULL");
  if (!h_params) return fail(ctx, MORSE_EINVAL, "h_params is NULL");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(h_params[k])) return fail(ctx, MORSE_EINVAL, "trajectory parameters must be finite");
  if (!(h_params[2] > 0.0)) return fail(ctx, MORSE_EINVAL, "tE must be > 0");
  if (n < 0) return fail(ctx, MORSE_EINVAL, "n < 0");
  if (n == 0) return MORSE_OK;
  if (!d_t || !d_zeta) return fail(ctx, MORSE_EINVAL, "d_t / d_zeta is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_traj_positions(d_t, n, h_params[0], h_params[1], h_params[2], h_params[3],
                                     d_zeta, ctx->stream));
  return MORSE_OK;
}

}  // extern "C"
