// Entry points whose implementation is not built yet: they validate nothing and report it.
#include "common.h"

using namespace dpm;

namespace dpm {
dpm_status launch_bf16x3_pass(int, AxisKind, bool, InKind, OutKind, const PassArgs&, const Plan*,
                              int, hipStream_t) {
  set_error("DPM_BF16X3: not available in this build");
  return DPM_EINVAL;
}
}  // namespace dpm
