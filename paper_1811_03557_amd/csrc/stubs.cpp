// Entry points whose implementation is not built yet: they validate nothing and report it.
#include "common.h"

using namespace dpm;

extern "C" {
dpm_status dpm_build_boundary_matrix(const dpm_grid*, const uint8_t*, int32_t, const double*,
                                     const dpm_opts*, void*, dpm_bep**, double*) {
  set_error("dpm_build_boundary_matrix: not available in this build");
  return DPM_EINVAL;
}
dpm_status dpm_bep_info(const dpm_bep*, int32_t*, int32_t*, int32_t*, double*, double*) {
  set_error("dpm_bep_info: not available in this build");
  return DPM_EINVAL;
}
dpm_status dpm_bep_solve(const dpm_bep*, int32_t, const double*, double*, void*) {
  set_error("dpm_bep_solve: not available in this build");
  return DPM_EINVAL;
}
dpm_status dpm_step_workspace_size(const dpm_bep*, const dpm_opts*, size_t*) {
  set_error("dpm_step_workspace_size: not available in this build");
  return DPM_EINVAL;
}
dpm_status dpm_step(const dpm_bep*, double, double, const double*, const double*, double*,
                    double*, const dpm_opts*, void*, dpm_info*) {
  set_error("dpm_step: not available in this build");
  return DPM_EINVAL;
}
dpm_status dpm_gauss_state(const dpm_bep*, const dpm_geometry*, double, double, const double*,
                           double*, void*) {
  set_error("dpm_gauss_state: not available in this build");
  return DPM_EINVAL;
}
void dpm_bep_destroy(dpm_bep*) {}
}
namespace dpm {
dpm_status launch_bf16x3_pass(int, AxisKind, bool, InKind, OutKind, const PassArgs&, const Plan*,
                              int, hipStream_t) {
  set_error("DPM_BF16X3: not available in this build");
  return DPM_EINVAL;
}
}  // namespace dpm
