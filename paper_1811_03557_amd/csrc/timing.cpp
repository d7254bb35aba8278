// Measurement support: hipEvents around the sweep launches of sampled chunks while enabled
// (dpm_timing_begin / dpm_timing_end).  A chunk of right-hand sides [rhs0, rhs0 + nb) is sampled
// when it holds an index that is a multiple of the stride, so a benchmark can time a few chunks
// of every batch without an event pair around each of its launches.  Process-wide and not
// thread safe: meant for a benchmark driving one stream.
#include <vector>

#include "common.h"

namespace dpm {

namespace {
struct TimingState {
  bool on = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> kind;
  size_t used = 0;             // events used
  int stride = 1;
};
TimingState g_tm;
}  // namespace

bool timing_enabled() { return g_tm.on; }

bool timing_on(int rhs0, int nb) {
  if (!g_tm.on || g_tm.used + 2 > g_tm.ev.size()) return false;
  const int st = g_tm.stride;
  const int first = (rhs0 + st - 1) / st;  // smallest multiple index >= rhs0
  return (long long)first * st < (long long)rhs0 + nb;
}

void timing_before(hipStream_t s) { (void)hipEventRecord(g_tm.ev[g_tm.used], s); }

void timing_after(hipStream_t s, int kind) {
  (void)hipEventRecord(g_tm.ev[g_tm.used + 1], s);
  g_tm.kind.push_back(kind);
  g_tm.used += 2;
}

}  // namespace dpm

using namespace dpm;

extern "C" {

dpm_status dpm_timing_begin(int32_t max_launches, int32_t rhs_stride) {
  clear_error();
  if (max_launches <= 0 || max_launches > (1 << 20)) { set_error("max_launches out of range"); return DPM_EINVAL; }
  if (rhs_stride <= 0) { set_error("rhs_stride must be > 0"); return DPM_EINVAL; }
  for (hipEvent_t e : g_tm.ev) (void)hipEventDestroy(e);
  g_tm = TimingState();
  g_tm.ev.resize(2 * (size_t)max_launches);
  for (auto& e : g_tm.ev) DPM_TRY_HIP(hipEventCreate(&e));
  g_tm.kind.reserve(max_launches);
  g_tm.stride = rhs_stride;
  g_tm.on = true;
  return DPM_OK;
}

dpm_status dpm_timing_end(int32_t nkinds, int32_t* counts, double* mean_ms) {
  clear_error();
  if (!g_tm.on) { set_error("timing was not started"); return DPM_EINVAL; }
  if (nkinds <= 0 || !counts || !mean_ms) { set_error("bad output arrays"); return DPM_EINVAL; }
  for (int k = 0; k < nkinds; ++k) { counts[k] = 0; mean_ms[k] = 0.0; }
  dpm_status st = DPM_OK;
  for (size_t i = 0; i < g_tm.kind.size(); ++i) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(g_tm.ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_tm.ev[2 * i], g_tm.ev[2 * i + 1]);
    if (e != hipSuccess) { set_error("event timing failed: %s", hipGetErrorString(e)); st = DPM_EHIP; break; }
    const int k = g_tm.kind[i];
    if (k < nkinds) { counts[k] += 1; mean_ms[k] += ms; }
  }
  for (int k = 0; k < nkinds; ++k) if (counts[k] > 0) mean_ms[k] /= counts[k];
  for (hipEvent_t e : g_tm.ev) (void)hipEventDestroy(e);
  g_tm = TimingState();
  return st;
}

}  // extern "C"
