// Host-only checks of the library's argument validation (no device is touched):
// built by tests/test_host_validation.py with hipcc for the host only.
#include "../paper_1511_01157_amd/csrc/host.h"

#include <cstdio>

using namespace morse::host;

namespace morse {
namespace host {
thread_local std::string g_thread_error;  // defined by the library's api_ctx.hip
}  // namespace host
}  // namespace morse

static int lc_status(const int64_t* off, int n_events) {
  static const double tref[4] = {0.0, 0.0, 0.0, 0.0};
  morse_ctx ctx;
  morse_lightcurves lc{};
  lc.n_events = n_events;
  lc.h_offsets = off;
  lc.h_t_ref = tref;
  // device pointers are only tested for NULL on the host
  lc.d_t = reinterpret_cast<const float*>(0x1000);
  lc.d_flux = reinterpret_cast<const double*>(0x2000);
  lc.d_weight = reinterpret_cast<const double*>(0x3000);
  return check_lightcurves(&ctx, &lc);
}

int main() {
  const int64_t cap = kMaxEventPoints;
  const int64_t ok[3] = {0, 3, 3 + cap};
  const int64_t too_long[3] = {0, 3, 4 + cap};
  const int64_t too_short[3] = {0, 3, 5};
  const int64_t bad_start[3] = {1, 4, 8};
  std::printf("%d %d %d %d %lld\n", lc_status(ok, 2), lc_status(too_long, 2),
              lc_status(too_short, 2), lc_status(bad_start, 2), (long long)cap);
  return 0;
}
