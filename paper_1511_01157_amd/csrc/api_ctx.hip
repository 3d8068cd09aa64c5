// C ABI of the gfx950 map-build / trajectory-search library (include/morse.h):
// version, errors, contexts (device, stream, workspace) and kernel timing.

#include "host.h"

using namespace morse;
using namespace morse::host;

namespace morse {
namespace host {
thread_local std::string g_thread_error;
}  // namespace host
}  // namespace morse

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
  if (hipStreamCreate(&c->capture_stream) != hipSuccess ||
      // non-blocking, default priority: ordered against the context's stream by the
      // refinement's own fork and join events only, also when that is the null stream
      hipStreamCreateWithFlags(&c->fork_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess) {
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->fork_stream) (void)hipStreamDestroy(c->fork_stream);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(nullptr, MORSE_EHIP, "stream or event creation failed");
  }
  // the allocation-free entry point's scratch address on this device, looked up once
  char* scratch = nullptr;
  const int rc = noalloc_scratch(device, &scratch);
  if (rc != MORSE_OK) {
    morse_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return MORSE_OK;
}

int morse_ctx_destroy(morse_ctx* ctx) {
  if (!ctx) return MORSE_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamSynchronize(ctx->fork_stream);  // before the workspace it reads is freed
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->refine_gexec) (void)hipGraphExecDestroy(ctx->refine_gexec);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->aux) (void)hipFree(ctx->aux);
  if (ctx->taps) (void)hipFree(ctx->taps);
  if (ctx->smeta.p) (void)hipFree(ctx->smeta.p);
  if (ctx->cmeta.p) (void)hipFree(ctx->cmeta.p);
  for (MetaBuf* mb : {&ctx->stack_taps, &ctx->fft_tw, &ctx->fft_spec, &ctx->lmeta, &ctx->fs_crit})
    if (mb->p) (void)hipFree(mb->p);
  for (const auto& t : ctx->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
  (void)hipEventDestroy(ctx->join_ev);
  (void)hipEventDestroy(ctx->fork_ev);
  (void)hipStreamDestroy(ctx->fork_stream);
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

}  // extern "C"
