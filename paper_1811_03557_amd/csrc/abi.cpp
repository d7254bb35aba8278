// extern "C" entry points of libdpm: argument validation, then the internal implementation.
// Nothing is enqueued when validation fails.
#include <cmath>

#include "common.h"

namespace dpm {
const char* last_error_text();
dpm_status classify_impl(const dpm_grid& g, const dpm_geometry& geo, uint8_t* m_plus, hipStream_t s);
dpm_status gamma_points_impl(const dpm_grid& g, const uint8_t* m_plus, int32_t* n_gamma,
                             int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, hipStream_t s);
dpm_status basis_impl(const dpm_grid& g, const dpm_geometry& geo, int32_t n_gamma,
                      const int32_t* idx, int32_t lmax, int32_t beta, double* basis, double* d_out,
                      hipStream_t s);
dpm_status validate_geometry(const dpm_geometry* geo);
}  // namespace dpm

using namespace dpm;

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

extern "C" {

const char* dpm_last_error(void) { return last_error_text(); }

dpm_status dpm_prepare(int32_t n) {
  clear_error();
  if (!fft_size_supported(n)) {
    set_error("n = %d: n + 1 must be a power of two with 7 <= n <= 1023", n);
    return DPM_EINVAL;
  }
  const Plan* p = nullptr;
  return get_plan(n, &p);
}

dpm_status dpm_workspace_size(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts,
                              size_t* bytes) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (!bytes) { set_error("bytes is NULL"); return DPM_EINVAL; }
  return workspace_size_impl(*grid, nrhs, *opts, bytes);
}

dpm_status aux_solve_batched(const dpm_grid* grid, int32_t nrhs, const void* b, void* u,
                             const dpm_opts* opts, void* stream, dpm_info* info) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (!b || !u) { set_error("b or u is NULL"); return DPM_EINVAL; }
  if (!aligned16(b) || !aligned16(u) || !aligned16(opts->workspace)) {
    set_error("b, u and workspace must be 16-byte aligned");
    return DPM_EINVAL;
  }
  const size_t bytes = (size_t)nrhs * grid->n * grid->n * grid->n * (opts->io_fp64 ? 8 : 4);
  const char* bb = static_cast<const char*>(b);
  const char* ub = static_cast<const char*>(u);
  if (bb < ub + bytes && ub < bb + bytes) { set_error("b and u overlap"); return DPM_EINVAL; }
  return aux_solve_impl(*grid, nrhs, b, u, *opts, static_cast<hipStream_t>(stream), info);
}

dpm_status aux_solve(const dpm_grid* grid, const void* b, void* u, const dpm_opts* opts,
                     void* stream, dpm_info* info) {
  return aux_solve_batched(grid, 1, b, u, opts, stream, info);
}

dpm_status dpm_classify(const dpm_grid* grid, const dpm_geometry* geom, uint8_t* m_plus,
                        void* stream) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_geometry(geom));
  if (!m_plus) { set_error("m_plus is NULL"); return DPM_EINVAL; }
  return classify_impl(*grid, *geom, m_plus, static_cast<hipStream_t>(stream));
}

dpm_status dpm_gamma_points(const dpm_grid* grid, const uint8_t* m_plus, int32_t* n_gamma,
                            int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, void* stream) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  if (!m_plus || !n_gamma || !n_gamma_in) { set_error("m_plus or a count pointer is NULL"); return DPM_EINVAL; }
  if ((idx == nullptr) != (is_in == nullptr)) { set_error("idx and is_in must both be given or both NULL"); return DPM_EINVAL; }
  return gamma_points_impl(*grid, m_plus, n_gamma, n_gamma_in, idx, is_in,
                           static_cast<hipStream_t>(stream));
}

dpm_status dpm_basis(const dpm_grid* grid, const dpm_geometry* geom, int32_t n_gamma,
                     const int32_t* idx, int32_t lmax, int32_t beta, double* basis,
                     double* d_out, void* stream) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_geometry(geom));
  if (n_gamma <= 0 || !idx || !basis) { set_error("empty gamma or NULL pointer"); return DPM_EINVAL; }
  if (lmax < 0 || lmax > 40) { set_error("lmax out of range [0, 40]"); return DPM_EINVAL; }
  if (beta != 0 && beta != 1) { set_error("beta must be 0 or 1"); return DPM_EINVAL; }
  if (!aligned16(basis)) { set_error("basis must be 16-byte aligned"); return DPM_EINVAL; }
  return basis_impl(*grid, *geom, n_gamma, idx, lmax, beta, basis, d_out,
                    static_cast<hipStream_t>(stream));
}

}  // extern "C"
