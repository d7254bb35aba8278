// extern "C" entry points of libdpm: argument validation, then the internal implementation.
// Nothing is enqueued when validation fails.
#include <cmath>

#include "bep.h"

namespace dpm {
const char* last_error_text();
dpm_status classify_impl(const dpm_grid& g, const dpm_geometry& geo, uint8_t* m_plus, hipStream_t s);
dpm_status gamma_points_impl(const dpm_grid& g, const uint8_t* m_plus, int32_t* n_gamma,
                             int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, hipStream_t s);
dpm_status basis_impl(const dpm_grid& g, const dpm_geometry& geo, int32_t n_gamma,
                      const int32_t* idx, int32_t lmax, int32_t beta, double* basis, double* d_out,
                      hipStream_t s);
dpm_status basis_zonal_impl(const dpm_grid& g, const dpm_geometry& geo, int32_t n_gamma,
                            const int32_t* idx, int32_t mmax, int32_t beta, double* basis,
                            double* d_out, hipStream_t s);
dpm_status validate_geometry(const dpm_geometry* geo);
dpm_status step_workspace_impl(const dpm_bep* b, const dpm_opts& o, size_t* bytes);
dpm_status step_impl(const dpm_bep* b, double dt, double chi, const double* rho_in,
                     const double* c_in, double* rho_out, double* c_out, const dpm_opts& o,
                     hipStream_t s, dpm_info* info);
dpm_status stepper_create_impl(const dpm_bep* b, double dt, double chi, double* rho, double* c,
                               const dpm_opts& o, hipStream_t s, dpm_stepper** out);
dpm_status stepper_run_impl(dpm_stepper* p, int nsteps, hipStream_t s);
dpm_status stepper_first_nonfinite_impl(const dpm_stepper* p, hipStream_t s, int32_t* step);
void stepper_destroy_impl(dpm_stepper* p);
dpm_status gauss_state_impl(const dpm_bep* b, const dpm_geometry& geo, double amp, double rate,
                            const double* c3, double* out, hipStream_t s);
dpm_status dd_build_impl(const dpm_dd_params& prm, const dpm_opts& o, hipStream_t s,
                         dpm_dd** out, double* A_out);
dpm_status dd_step_workspace_impl(const dpm_dd* d, const dpm_opts& o, size_t* bytes);
dpm_status dd_step_impl(const dpm_dd* d, double dt, double chi, const double* const in[4],
                        double* const out[4], const dpm_opts& o, hipStream_t s);
dpm_status dd_masks_impl(const dpm_dd* d, int l, uint8_t* m_plus, uint8_t* n_plus, hipStream_t s);
dpm_status dd_gauss_impl(const dpm_dd* d, int l, double amp, double rate, const double c0[3],
                         double* out, hipStream_t s);
void dd_destroy(dpm_dd* d);
double dd_sigma(const dpm_dd* d);
size_t diag_workspace_bytes();
dpm_status diagnostics_impl(const dpm_bep* b, const double* rho, const double* c, double* out3,
                            void* ws, hipStream_t s);
dpm_status dd_diagnostics_impl(const dpm_dd* d, const double* const state[4], double* out3,
                               void* ws, hipStream_t s);
dpm_status dd_info_impl(const dpm_dd* d, int32_t n_gamma[2], int32_t n_in[2], int32_t n_rows[2],
                        int32_t* n_cols, double* rmin, double* rmax);
dpm_status dd_lsq_info_impl(const dpm_dd* d, double* rcond, int32_t* rank, double* smin_ratio);
int dd_lsq_method(const dpm_dd* d);
dpm_status dd2_build_impl(const dpm_dd2_params& prm, const dpm_opts& o, hipStream_t s,
                          dpm_dd** out, double* A_out);
dpm_status dd_rebuild_impl(dpm_dd* d, double sigma, hipStream_t s, void* scratch, size_t bytes);
size_t dd_rebuild_workspace_bytes(const dpm_dd* d);
dpm_status dd_run_workspace_impl(const dpm_dd* d, const dpm_opts& o, size_t* bytes);
dpm_status dd_stepper_create_impl(const dpm_dd* d, double dt, double chi, double* const state[4],
                                  const dpm_opts& o, void** out);
dpm_status dd_stepper_run_impl(void* h, int nsteps, hipStream_t s);
void dd_stepper_destroy_impl(void* h);
dpm_status dd_run_impl(dpm_dd* d, const dpm_run_params& p, double* const state[4],
                       const dpm_opts& o, hipStream_t s, dpm_run_info* info, double* dt_hist,
                       uint8_t* rebuilt_hist);
}  // namespace dpm

using namespace dpm;

static bool aligned_to(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }
static bool aligned16(const void* p) { return aligned_to(p, 16); }

extern "C" {

const char* dpm_last_error(void) { return last_error_text(); }

dpm_status dpm_prepare(int32_t n) {
  clear_error();
  if (!fft_size_supported(n) && !dense_size_supported(n) && !blue_size_supported(n)) {
    set_error("n = %d: no transform for this size (n + 1 a power of two up to 1023, "
              "7 <= n <= %d for DPM_FP64, 7 <= n <= %d for DPM_FP64_GEMM)", n, kBlueMaxN,
              kDenseMaxN);
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

dpm_status dpm_rhs_chunk(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts, int32_t* chunk) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (!chunk) { set_error("chunk is NULL"); return DPM_EINVAL; }
  *chunk = rhs_chunk_of(*grid, nrhs, *opts);
  return DPM_OK;
}

dpm_status dpm_autotune(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts, const void* b,
                        void* u, int32_t reps, void* stream, int32_t* widths, int32_t* sweeps,
                        int32_t* zcols, double* ms, int32_t* count, int32_t* best,
                        int32_t* best_sweeps, int32_t* best_zcols) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (reps < 1 || reps > 100) { set_error("reps must be in [1, 100]"); return DPM_EINVAL; }
  if (!b || !u) { set_error("b or u is NULL"); return DPM_EINVAL; }
  if (!aligned_to(b, opts->io_fp64 ? 8 : 4) || !aligned_to(u, opts->io_fp64 ? 8 : 4) ||
      !aligned16(opts->workspace)) {
    set_error("b and u must be aligned to their element size, the workspace to 16 bytes");
    return DPM_EINVAL;
  }
  const size_t bytes = (size_t)nrhs * grid->n * grid->n * grid->n * (opts->io_fp64 ? 8 : 4);
  const char* bb = static_cast<const char*>(b);
  const char* ub = static_cast<const char*>(u);
  if (bb < ub + bytes && ub < bb + bytes) { set_error("b and u overlap"); return DPM_EINVAL; }
  return autotune_impl(*grid, nrhs, *opts, b, u, reps, static_cast<hipStream_t>(stream), widths,
                       sweeps, zcols, ms, count, best, best_sweeps, best_zcols);
}

void dpm_autotune_reset(void) { autotune_reset(); }

dpm_status aux_solve_batched(const dpm_grid* grid, int32_t nrhs, const void* b, void* u,
                             const dpm_opts* opts, void* stream, dpm_info* info) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (!b || !u) { set_error("b or u is NULL"); return DPM_EINVAL; }
  if (!aligned_to(b, opts->io_fp64 ? 8 : 4) || !aligned_to(u, opts->io_fp64 ? 8 : 4) ||
      !aligned16(opts->workspace)) {
    set_error("b and u must be aligned to their element size, the workspace to 16 bytes");
    return DPM_EINVAL;
  }
  const size_t bytes = (size_t)nrhs * grid->n * grid->n * grid->n * (opts->io_fp64 ? 8 : 4);
  const char* bb = static_cast<const char*>(b);
  const char* ub = static_cast<const char*>(u);
  if (bb < ub + bytes && ub < bb + bytes) { set_error("b and u overlap"); return DPM_EINVAL; }
  return aux_solve_impl(*grid, nrhs, b, u, *opts, static_cast<hipStream_t>(stream), info);
}

dpm_status aux_solve_batched_sigma(const dpm_grid* grid, int32_t nrhs, const double* sigma,
                                   const void* b, void* u, const dpm_opts* opts, void* stream,
                                   dpm_info* info) {
  clear_error();
  if (!sigma) { set_error("sigma is NULL"); return DPM_EINVAL; }
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  for (int i = 0; i < nrhs; ++i)
    if (!(sigma[i] >= 0.0) || !std::isfinite(sigma[i])) {
      set_error("sigma[%d] must be finite and >= 0", i);
      return DPM_EINVAL;
    }
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (!b || !u) { set_error("b or u is NULL"); return DPM_EINVAL; }
  if (!aligned_to(b, opts->io_fp64 ? 8 : 4) || !aligned_to(u, opts->io_fp64 ? 8 : 4) ||
      !aligned16(opts->workspace)) {
    set_error("b and u must be aligned to their element size, the workspace to 16 bytes");
    return DPM_EINVAL;
  }
  const size_t bytes = (size_t)nrhs * grid->n * grid->n * grid->n * (opts->io_fp64 ? 8 : 4);
  const char* bb = static_cast<const char*>(b);
  const char* ub = static_cast<const char*>(u);
  if (bb < ub + bytes && ub < bb + bytes) { set_error("b and u overlap"); return DPM_EINVAL; }
  return aux_solve_impl(*grid, nrhs, b, u, *opts, static_cast<hipStream_t>(stream), info, sigma);
}

dpm_status aux_solve_batched_noalloc(const dpm_grid* grid, int32_t nrhs, const void* b, void* u,
                                     const dpm_opts* opts, void* stream, dpm_info* info) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (nrhs <= 0) { set_error("nrhs must be > 0"); return DPM_EINVAL; }
  if (!b || !u) { set_error("b or u is NULL"); return DPM_EINVAL; }
  if (!aligned_to(b, opts->io_fp64 ? 8 : 4) || !aligned_to(u, opts->io_fp64 ? 8 : 4)) {
    set_error("b and u must be aligned to their element size");
    return DPM_EINVAL;
  }
  const size_t bytes = (size_t)nrhs * grid->n * grid->n * grid->n * (opts->io_fp64 ? 8 : 4);
  const char* bb = static_cast<const char*>(b);
  const char* ub = static_cast<const char*>(u);
  if (bb < ub + bytes && ub < bb + bytes) { set_error("b and u overlap"); return DPM_EINVAL; }
  // size check on the host before any device call: the static scratch must hold the
  // per-right-hand-side state and at least one right-hand side per launch
  dpm_opts o = *opts;
  o.workspace = nullptr;
  o.workspace_bytes = kStaticScratchBytes;
  // the library's layout choice takes the per-axis sweeps when the split layout's separator
  // planes do not fit beside the rest
  if (o.sweeps == DPM_SWEEPS_AUTO && workspace_for_chunk(*grid, nrhs, o, 1) > kStaticScratchBytes)
    o.sweeps = DPM_SWEEPS_AXIS;
  if (workspace_for_chunk(*grid, nrhs, o, 1) > kStaticScratchBytes) {
    set_error("aux_solve_batched_noalloc: n = %d, nrhs = %d needs %zu bytes of scratch, more "
              "than the static maximum of %zu", grid->n, nrhs, workspace_for_chunk(*grid, nrhs, o, 1),
              kStaticScratchBytes);
    return DPM_EINVAL;
  }
  if (o.rhs_chunk > 0 && workspace_for_chunk(*grid, nrhs, o, o.rhs_chunk) > kStaticScratchBytes) {
    set_error("aux_solve_batched_noalloc: rhs_chunk = %d does not fit the static scratch of %zu "
              "bytes", o.rhs_chunk, kStaticScratchBytes);
    return DPM_EINVAL;
  }
  DPM_TRY(static_scratch(&o.workspace));
  return aux_solve_impl(*grid, nrhs, b, u, o, static_cast<hipStream_t>(stream), info, nullptr,
                        true);
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

dpm_status dpm_basis_zonal(const dpm_grid* grid, const dpm_geometry* geom, int32_t n_gamma,
                           const int32_t* idx, int32_t mmax, int32_t beta, double* basis,
                           double* d_out, void* stream) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_geometry(geom));
  if (n_gamma <= 0 || !idx || !basis) { set_error("empty gamma or NULL pointer"); return DPM_EINVAL; }
  if (mmax < 0 || mmax > 1023) { set_error("mmax out of range [0, 1023]"); return DPM_EINVAL; }
  if (beta != 0 && beta != 1) { set_error("beta must be 0 or 1"); return DPM_EINVAL; }
  if (!aligned_to(basis, 8) || (d_out && !aligned_to(d_out, 8))) {
    set_error("basis and d_out must be 8-byte aligned");
    return DPM_EINVAL;
  }
  return basis_zonal_impl(*grid, *geom, n_gamma, idx, mmax, beta, basis, d_out,
                          static_cast<hipStream_t>(stream));
}

dpm_status dpm_build_boundary_matrix(const dpm_grid* grid, const uint8_t* m_plus,
                                     int32_t n_basis, const double* basis, const dpm_opts* opts,
                                     void* stream, dpm_bep** out, double* A_out) {
  clear_error();
  DPM_TRY(validate_grid(grid));
  DPM_TRY(validate_opts(*grid, opts));
  if (!m_plus || !basis || !out) { set_error("m_plus, basis or out is NULL"); return DPM_EINVAL; }
  if (n_basis <= 0 || n_basis > 1024) { set_error("n_basis out of range [1, 1024]"); return DPM_EINVAL; }
  if (!opts->io_fp64) { set_error("the boundary matrix needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  *out = nullptr;
  return build_bep_impl(*grid, m_plus, n_basis, basis, *opts, static_cast<hipStream_t>(stream),
                        out, A_out);
}

dpm_status dpm_bep_info(const dpm_bep* bep, int32_t* n_gamma, int32_t* n_gamma_in,
                        int32_t* n_basis, double* min_abs_rdiag, double* max_abs_rdiag) {
  clear_error();
  if (!bep) { set_error("bep is NULL"); return DPM_EINVAL; }
  if (n_gamma) *n_gamma = bep->n_gamma;
  if (n_gamma_in) *n_gamma_in = bep->n_in;
  if (n_basis) *n_basis = bep->n_basis;
  if (min_abs_rdiag) *min_abs_rdiag = bep->rdiag_min;
  if (max_abs_rdiag) *max_abs_rdiag = bep->rdiag_max;
  return DPM_OK;
}

dpm_status dpm_bep_device_bytes(const dpm_bep* bep, size_t* bytes) {
  clear_error();
  if (!bep || !bytes) { set_error("bep or bytes is NULL"); return DPM_EINVAL; }
  const size_t v = (size_t)bep->grid.n * bep->grid.n * bep->grid.n;
  const size_t ng = (size_t)bep->n_gamma, ni = (size_t)bep->n_in, nb = (size_t)bep->n_basis;
  *bytes = 2 * v                      // M+ and N+ masks
           + sizeof(int32_t) * v      // node -> gamma position map
           + (sizeof(int32_t) + 1) * ng + 2 * sizeof(int32_t) * ni  // gamma lists
           + sizeof(double) * (nb * ng + 2 * nb * ni + nb);         // basis, A, P, tau
  return DPM_OK;
}

dpm_status dpm_bep_solve(const dpm_bep* bep, int32_t nvec, const double* g, double* C,
                         void* stream) {
  clear_error();
  if (!bep || !g || !C) { set_error("bep, g or C is NULL"); return DPM_EINVAL; }
  if (nvec <= 0 || nvec > 65535) { set_error("nvec out of range"); return DPM_EINVAL; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  qr_solve(bep, nvec, g, C, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { set_error("dpm_bep_solve: %s", hipGetErrorString(e)); return DPM_EHIP; }
  return DPM_OK;
}

dpm_status dpm_step_workspace_size(const dpm_bep* bep, const dpm_opts* opts, size_t* bytes) {
  clear_error();
  if (!bep || !bytes) { set_error("bep or bytes is NULL"); return DPM_EINVAL; }
  DPM_TRY(validate_opts(bep->grid, opts));
  return step_workspace_impl(bep, *opts, bytes);
}

dpm_status dpm_step(const dpm_bep* bep, double dt, double chi, const double* rho_in,
                    const double* c_in, double* rho_out, double* c_out, const dpm_opts* opts,
                    void* stream, dpm_info* info) {
  clear_error();
  if (!bep || !rho_in || !c_in || !rho_out || !c_out || !opts) { set_error("NULL argument"); return DPM_EINVAL; }
  // pointer checks first (they need nothing from the handle)
  if (!aligned_to(rho_in, 8) || !aligned_to(c_in, 8) || !aligned_to(rho_out, 8) ||
      !aligned_to(c_out, 8) || !aligned16(opts->workspace)) {
    set_error("the state volumes must be 8-byte aligned, the workspace 16-byte aligned");
    return DPM_EINVAL;
  }
  // the outputs are written after every read of the inputs, so they may alias them, but both
  // species are written by one kernel
  if (rho_out == c_out) { set_error("rho_out and c_out must be different buffers"); return DPM_EINVAL; }
  DPM_TRY(validate_opts(bep->grid, opts));
  if (!opts->io_fp64) { set_error("dpm_step needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(chi)) { set_error("dt must be finite and > 0, chi finite"); return DPM_EINVAL; }
  if (std::fabs(bep->grid.sigma * dt - 1.0) > 1e-12) {
    set_error("the handle was built with sigma = %g but 1/dt = %g", bep->grid.sigma, 1.0 / dt);
    return DPM_EINVAL;
  }
  return step_impl(bep, dt, chi, rho_in, c_in, rho_out, c_out, *opts,
                   static_cast<hipStream_t>(stream), info);
}

dpm_status dpm_stepper_create(const dpm_bep* bep, double dt, double chi, double* rho, double* c,
                              const dpm_opts* opts, void* stream, dpm_stepper** out) {
  clear_error();
  if (!bep || !rho || !c || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  *out = nullptr;
  DPM_TRY(validate_opts(bep->grid, opts));
  if (!opts->io_fp64) { set_error("dpm_stepper_create needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!aligned_to(rho, 8) || !aligned_to(c, 8) || !aligned16(opts->workspace)) {
    set_error("rho and c must be 8-byte aligned, the workspace 16-byte aligned");
    return DPM_EINVAL;
  }
  if (rho == c) { set_error("rho and c must be different buffers"); return DPM_EINVAL; }
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(chi)) { set_error("dt must be finite and > 0, chi finite"); return DPM_EINVAL; }
  if (std::fabs(bep->grid.sigma * dt - 1.0) > 1e-12) {
    set_error("the handle was built with sigma = %g but 1/dt = %g", bep->grid.sigma, 1.0 / dt);
    return DPM_EINVAL;
  }
  return stepper_create_impl(bep, dt, chi, rho, c, *opts, static_cast<hipStream_t>(stream), out);
}

dpm_status dpm_stepper_run(dpm_stepper* st, int32_t nsteps, void* stream) {
  clear_error();
  if (!st) { set_error("stepper is NULL"); return DPM_EINVAL; }
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return DPM_EINVAL; }
  return stepper_run_impl(st, nsteps, static_cast<hipStream_t>(stream));
}

dpm_status dpm_stepper_first_nonfinite(const dpm_stepper* st, void* stream, int32_t* step) {
  clear_error();
  if (!st || !step) { set_error("stepper or step is NULL"); return DPM_EINVAL; }
  return stepper_first_nonfinite_impl(st, static_cast<hipStream_t>(stream), step);
}

void dpm_stepper_destroy(dpm_stepper* st) { stepper_destroy_impl(st); }

dpm_status dpm_cfl_scan(const dpm_bep* bep, const double* rho, const double* c, double* out2,
                        void* stream) {
  clear_error();
  if (!bep || !rho || !c || !out2) { set_error("NULL argument"); return DPM_EINVAL; }
  if (!aligned_to(rho, 8) || !aligned_to(c, 8) || !aligned_to(out2, 8)) {
    set_error("rho, c and out2 must be 8-byte aligned");
    return DPM_EINVAL;
  }
  return cfl_scan_impl(bep, rho, c, out2, static_cast<hipStream_t>(stream));
}

dpm_status dpm_bep_rebuild_workspace_size(const dpm_bep* bep, size_t* bytes) {
  clear_error();
  if (!bep || !bytes) { set_error("bep or bytes is NULL"); return DPM_EINVAL; }
  *bytes = rebuild_scratch_bytes(bep);
  return DPM_OK;
}

dpm_status dpm_bep_rebuild(dpm_bep* bep, double sigma, void* workspace, size_t workspace_bytes,
                           void* stream) {
  clear_error();
  if (!bep) { set_error("bep is NULL"); return DPM_EINVAL; }
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) { set_error("sigma must be finite and >= 0"); return DPM_EINVAL; }
  if (!aligned16(workspace)) { set_error("the workspace must be 16-byte aligned"); return DPM_EINVAL; }
  return rebuild_bep_impl(bep, sigma, static_cast<hipStream_t>(stream), workspace,
                          workspace_bytes);
}

dpm_status dpm_run_workspace_size(const dpm_bep* bep, const dpm_opts* opts, size_t* bytes) {
  clear_error();
  if (!bep || !bytes) { set_error("bep or bytes is NULL"); return DPM_EINVAL; }
  DPM_TRY(validate_opts(bep->grid, opts));
  return run_workspace_impl(bep, *opts, bytes);
}

dpm_status dpm_run(dpm_bep* bep, const dpm_run_params* params, double* rho, double* c,
                   const dpm_opts* opts, void* stream, dpm_run_info* info, double* dt_hist,
                   uint8_t* rebuilt_hist) {
  clear_error();
  if (!bep || !params || !rho || !c) { set_error("NULL argument"); return DPM_EINVAL; }
  DPM_TRY(validate_opts(bep->grid, opts));
  if (!opts->io_fp64) { set_error("dpm_run needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!aligned_to(rho, 8) || !aligned_to(c, 8) || !aligned16(opts->workspace)) {
    set_error("rho and c must be 8-byte aligned, the workspace 16-byte aligned");
    return DPM_EINVAL;
  }
  if (rho == c) { set_error("rho and c must be different buffers"); return DPM_EINVAL; }
  if (!(params->chi >= 0.0) || !std::isfinite(params->chi)) { set_error("chi must be finite and >= 0"); return DPM_EINVAL; }
  if (std::isnan(params->t_final) || std::isnan(params->rho_cap) || std::isnan(params->rho_jump_cap)) { set_error("t_final, rho_cap and rho_jump_cap must not be NaN"); return DPM_EINVAL; }
  if (params->max_steps < 0) { set_error("max_steps must be >= 0"); return DPM_EINVAL; }
  if (!(bep->grid.sigma > 0.0)) { set_error("the handle's sigma must be > 0 (sigma = 1/dt)"); return DPM_EINVAL; }
  return run_impl(bep, *params, rho, c, *opts, static_cast<hipStream_t>(stream), info, dt_hist,
                  rebuilt_hist);
}

dpm_status dpm_gauss_state(const dpm_bep* bep, const dpm_geometry* geom, double amp,
                           double rate, const double center[3], double* out, void* stream) {
  clear_error();
  if (!bep || !out || !center) { set_error("NULL argument"); return DPM_EINVAL; }
  DPM_TRY(validate_geometry(geom));
  return gauss_state_impl(bep, *geom, amp, rate, center, out, static_cast<hipStream_t>(stream));
}

void dpm_bep_destroy(dpm_bep* bep) { destroy_bep(bep); }

dpm_status dpm_dd_build(const dpm_dd_params* params, const dpm_opts* opts, void* stream,
                        dpm_dd** out, double* A_out) {
  clear_error();
  if (!params || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  *out = nullptr;
  const dpm_dd_params& p = *params;
  for (const dpm_grid* g : {&p.grid1, &p.grid2}) {
    DPM_TRY(validate_grid(g));
    DPM_TRY(validate_opts(*g, opts));
  }
  if (!opts->io_fp64) { set_error("the boundary matrix needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (p.grid1.sigma != p.grid2.sigma) { set_error("both meshes need the same sigma (= 1/dt)"); return DPM_EINVAL; }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p.center[i])) { set_error("center must be finite"); return DPM_EINVAL; }
  if (!(p.r_z > 0.0) || !(p.r_split > p.r_z) || !(p.r_gamma > p.r_split) || !std::isfinite(p.r_gamma)) {
    set_error("the radii must satisfy 0 < r_z < r_split < r_gamma (finite)");
    return DPM_EINVAL;
  }
  if (p.m_gamma < 0 || p.m_z < 0 || (p.beta != 0 && p.beta != 1)) {
    set_error("m_gamma, m_z must be >= 0 and beta 0 or 1");
    return DPM_EINVAL;
  }
  if ((p.beta + 1) * (p.m_gamma + 1) + 3 * (p.m_z + 1) > 1024) {
    set_error("more than 1024 columns");
    return DPM_EINVAL;
  }
  return dd_build_impl(p, *opts, static_cast<hipStream_t>(stream), out, A_out);
}

dpm_status dpm_dd2_build(const dpm_dd2_params* params, const dpm_opts* opts, void* stream,
                         dpm_dd** out, double* A_out) {
  clear_error();
  if (!params || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  *out = nullptr;
  const dpm_dd2_params& p = *params;
  for (const dpm_grid* g : {&p.grid1, &p.grid2}) {
    DPM_TRY(validate_grid(g));
    DPM_TRY(validate_opts(*g, opts));
  }
  if (!opts->io_fp64) { set_error("the boundary matrix needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (p.grid1.sigma != p.grid2.sigma) { set_error("both meshes need the same sigma (= 1/dt)"); return DPM_EINVAL; }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p.origin1[i]) || !std::isfinite(p.origin2[i])) { set_error("origins must be finite"); return DPM_EINVAL; }
  if (!(p.r_gamma > 0.0) || !(p.r_z > 0.0) || !std::isfinite(p.r_gamma) || !std::isfinite(p.r_z) ||
      !std::isfinite(p.q_z) || !(std::fabs(p.q_z) - p.r_z < p.r_gamma) || !(p.r_gamma < std::fabs(p.q_z) + p.r_z) ||
      !(p.q_z > 0.0)) {
    set_error("the radii must satisfy q_z > 0 and q_z - r_z < r_gamma < q_z + r_z (Z meets Gamma)");
    return DPM_EINVAL;
  }
  if (!(p.eps_layers > 0.0) || !std::isfinite(p.eps_layers)) { set_error("eps_layers must be finite and > 0"); return DPM_EINVAL; }
  if (p.m_gamma < 0 || p.m_z < 0 || (p.beta != 0 && p.beta != 1)) {
    set_error("m_gamma, m_z must be >= 0 and beta 0 or 1");
    return DPM_EINVAL;
  }
  if (!(p.rcond >= 0.0 && p.rcond < 1.0)) { set_error("rcond must be in [0, 1)"); return DPM_EINVAL; }
  if (p.rcond > 0.0 && !svd_shape((p.beta + 1) * (p.m_gamma + 1) + 3 * (p.m_z + 1)).ok) {
    set_error("rcond > 0 supports at most 640 columns");
    return DPM_EINVAL;
  }
  if ((p.beta + 1) * (p.m_gamma + 1) + 3 * (p.m_z + 1) > 1024) {
    set_error("more than 1024 columns");
    return DPM_EINVAL;
  }
  return dd2_build_impl(p, *opts, static_cast<hipStream_t>(stream), out, A_out);
}

dpm_status dpm_dd_info(const dpm_dd* dd, int32_t n_gamma[2], int32_t n_gamma_in[2],
                       int32_t n_rows[2], int32_t* n_cols, double* min_abs_rdiag,
                       double* max_abs_rdiag) {
  clear_error();
  if (!dd) { set_error("dd is NULL"); return DPM_EINVAL; }
  return dd_info_impl(dd, n_gamma, n_gamma_in, n_rows, n_cols, min_abs_rdiag, max_abs_rdiag);
}

dpm_status dpm_dd_lsq_info(const dpm_dd* dd, double* rcond, int32_t* rank, double* smin_ratio) {
  clear_error();
  if (!dd) { set_error("dd is NULL"); return DPM_EINVAL; }
  return dd_lsq_info_impl(dd, rcond, rank, smin_ratio);
}

dpm_status dpm_dd_lsq_method(const dpm_dd* dd, int32_t* method) {
  clear_error();
  if (!dd || !method) { set_error("dd or method is NULL"); return DPM_EINVAL; }
  *method = dd_lsq_method(dd);
  return DPM_OK;
}

dpm_status dpm_bep_lsq_method(const dpm_bep* bep, int32_t* method) {
  clear_error();
  if (!bep || !method) { set_error("bep or method is NULL"); return DPM_EINVAL; }
  *method = bep->lsq_method;
  return DPM_OK;
}

dpm_status dpm_dd_masks(const dpm_dd* dd, int32_t l, uint8_t* m_plus, uint8_t* n_plus,
                        void* stream) {
  clear_error();
  if (!dd) { set_error("dd is NULL"); return DPM_EINVAL; }
  if (l != 0 && l != 1) { set_error("subdomain index must be 0 or 1"); return DPM_EINVAL; }
  return dd_masks_impl(dd, l, m_plus, n_plus, static_cast<hipStream_t>(stream));
}

dpm_status dpm_dd_step_workspace_size(const dpm_dd* dd, const dpm_opts* opts, size_t* bytes) {
  clear_error();
  if (!dd || !opts || !bytes) { set_error("NULL argument"); return DPM_EINVAL; }
  return dd_step_workspace_impl(dd, *opts, bytes);
}

dpm_status dpm_dd_step(const dpm_dd* dd, double dt, double chi, const double* const in[4],
                       double* const out[4], const dpm_opts* opts, void* stream) {
  clear_error();
  if (!dd || !in || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  for (int i = 0; i < 4; ++i)
    if (!in[i] || !out[i] || !aligned_to(in[i], 8) || !aligned_to(out[i], 8)) {
      set_error("volume %d is NULL or not 8-byte aligned", i);
      return DPM_EINVAL;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (out[i] == out[j]) { set_error("the four outputs must be different buffers"); return DPM_EINVAL; }
  if (!opts) { set_error("opts is NULL"); return DPM_EINVAL; }
  if (!opts->io_fp64) { set_error("dpm_dd_step needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!aligned16(opts->workspace)) { set_error("the workspace must be 16-byte aligned"); return DPM_EINVAL; }
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(chi)) { set_error("dt must be finite and > 0, chi finite"); return DPM_EINVAL; }
  if (std::fabs(dd_sigma(dd) * dt - 1.0) > 1e-12) {
    set_error("the handle was built with sigma = %g but 1/dt = %g", dd_sigma(dd), 1.0 / dt);
    return DPM_EINVAL;
  }
  return dd_step_impl(dd, dt, chi, in, out, *opts, static_cast<hipStream_t>(stream));
}

dpm_status dpm_dd_gauss_state(const dpm_dd* dd, int32_t l, double amp, double rate,
                              const double c0[3], double* out, void* stream) {
  clear_error();
  if (!dd || !c0 || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  if (l != 0 && l != 1) { set_error("subdomain index must be 0 or 1"); return DPM_EINVAL; }
  return dd_gauss_impl(dd, l, amp, rate, c0, out, static_cast<hipStream_t>(stream));
}

dpm_status dpm_dd_stepper_create(const dpm_dd* dd, double dt, double chi, double* const state[4],
                                 const dpm_opts* opts, dpm_dd_stepper** out) {
  clear_error();
  if (!dd || !state || !opts || !out) { set_error("NULL argument"); return DPM_EINVAL; }
  *out = nullptr;
  for (int i = 0; i < 4; ++i)
    if (!state[i] || !aligned_to(state[i], 8)) { set_error("volume %d is NULL or not 8-byte aligned", i); return DPM_EINVAL; }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (state[i] == state[j]) { set_error("the four state volumes must be different buffers"); return DPM_EINVAL; }
  if (!opts->io_fp64) { set_error("dpm_dd_stepper_create needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!aligned16(opts->workspace)) { set_error("the workspace must be 16-byte aligned"); return DPM_EINVAL; }
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(chi)) { set_error("dt must be finite and > 0, chi finite"); return DPM_EINVAL; }
  if (std::fabs(dd_sigma(dd) * dt - 1.0) > 1e-12) {
    set_error("the handle was built with sigma = %g but 1/dt = %g", dd_sigma(dd), 1.0 / dt);
    return DPM_EINVAL;
  }
  void* h = nullptr;
  DPM_TRY(dd_stepper_create_impl(dd, dt, chi, state, *opts, &h));
  *out = static_cast<dpm_dd_stepper*>(h);
  return DPM_OK;
}

dpm_status dpm_dd_stepper_run(dpm_dd_stepper* st, int32_t nsteps, void* stream) {
  clear_error();
  if (!st) { set_error("stepper is NULL"); return DPM_EINVAL; }
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return DPM_EINVAL; }
  return dd_stepper_run_impl(st, nsteps, static_cast<hipStream_t>(stream));
}

void dpm_dd_stepper_destroy(dpm_dd_stepper* st) { dd_stepper_destroy_impl(st); }

dpm_status dpm_dd_rebuild_workspace_size(const dpm_dd* dd, size_t* bytes) {
  clear_error();
  if (!dd || !bytes) { set_error("dd or bytes is NULL"); return DPM_EINVAL; }
  *bytes = dd_rebuild_workspace_bytes(dd);
  return DPM_OK;
}

dpm_status dpm_dd_rebuild(dpm_dd* dd, double sigma, void* workspace, size_t workspace_bytes,
                          void* stream) {
  clear_error();
  if (!dd) { set_error("dd is NULL"); return DPM_EINVAL; }
  if (!(sigma > 0.0) || !std::isfinite(sigma)) { set_error("sigma must be finite and > 0"); return DPM_EINVAL; }
  if (!aligned16(workspace)) { set_error("the workspace must be 16-byte aligned"); return DPM_EINVAL; }
  return dd_rebuild_impl(dd, sigma, static_cast<hipStream_t>(stream), workspace, workspace_bytes);
}

dpm_status dpm_dd_run_workspace_size(const dpm_dd* dd, const dpm_opts* opts, size_t* bytes) {
  clear_error();
  if (!dd || !bytes || !opts) { set_error("NULL argument"); return DPM_EINVAL; }
  return dd_run_workspace_impl(dd, *opts, bytes);
}

dpm_status dpm_dd_run(dpm_dd* dd, const dpm_run_params* params, double* const state[4],
                      const dpm_opts* opts, void* stream, dpm_run_info* info, double* dt_hist,
                      uint8_t* rebuilt_hist) {
  clear_error();
  if (!dd || !params || !state || !opts) { set_error("NULL argument"); return DPM_EINVAL; }
  for (int i = 0; i < 4; ++i)
    if (!state[i] || !aligned_to(state[i], 8)) { set_error("volume %d is NULL or not 8-byte aligned", i); return DPM_EINVAL; }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (state[i] == state[j]) { set_error("the four state volumes must be different buffers"); return DPM_EINVAL; }
  if (!opts->io_fp64) { set_error("dpm_dd_run needs FP64 solves (io_fp64 = 1)"); return DPM_EINVAL; }
  if (!aligned16(opts->workspace)) { set_error("the workspace must be 16-byte aligned"); return DPM_EINVAL; }
  if (!(params->chi >= 0.0) || !std::isfinite(params->chi)) { set_error("chi must be finite and >= 0"); return DPM_EINVAL; }
  if (std::isnan(params->t_final) || std::isnan(params->rho_cap) || std::isnan(params->rho_jump_cap)) { set_error("t_final, rho_cap and rho_jump_cap must not be NaN"); return DPM_EINVAL; }
  if (params->max_steps < 0) { set_error("max_steps must be >= 0"); return DPM_EINVAL; }
  if (!(dd_sigma(dd) > 0.0)) { set_error("the handle's sigma must be > 0 (sigma = 1/dt)"); return DPM_EINVAL; }
  return dd_run_impl(dd, *params, state, *opts, static_cast<hipStream_t>(stream), info, dt_hist,
                     rebuilt_hist);
}

void dpm_dd_destroy(dpm_dd* dd) { dd_destroy(dd); }

static dpm_status check_diag_ws(void* ws, size_t bytes) {
  if (diag_workspace_bytes() > DPM_DIAG_WORKSPACE_BYTES) {
    set_error("internal: diagnostics scratch exceeds DPM_DIAG_WORKSPACE_BYTES");
    return DPM_EINVAL;
  }
  if (!ws || !aligned_to(ws, 8) || bytes < DPM_DIAG_WORKSPACE_BYTES) {
    set_error("the diagnostics need an 8-byte aligned workspace of %zu bytes (%zu given)",
              (size_t)DPM_DIAG_WORKSPACE_BYTES, bytes);
    return DPM_EINVAL;
  }
  return DPM_OK;
}

dpm_status dpm_diagnostics(const dpm_bep* bep, const double* rho, const double* c, double* out3,
                           void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (!bep || !rho || !c || !out3) { set_error("NULL argument"); return DPM_EINVAL; }
  if (!aligned_to(rho, 8) || !aligned_to(c, 8) || !aligned_to(out3, 8)) { set_error("volumes and out3 must be 8-byte aligned"); return DPM_EINVAL; }
  DPM_TRY(check_diag_ws(workspace, workspace_bytes));
  return diagnostics_impl(bep, rho, c, out3, workspace, static_cast<hipStream_t>(stream));
}

dpm_status dpm_dd_diagnostics(const dpm_dd* dd, const double* const state[4], double* out3,
                              void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (!dd || !state || !out3) { set_error("NULL argument"); return DPM_EINVAL; }
  for (int i = 0; i < 4; ++i)
    if (!state[i] || !aligned_to(state[i], 8)) { set_error("volume %d is NULL or not 8-byte aligned", i); return DPM_EINVAL; }
  if (!aligned_to(out3, 8)) { set_error("out3 must be 8-byte aligned"); return DPM_EINVAL; }
  DPM_TRY(check_diag_ws(workspace, workspace_bytes));
  return dd_diagnostics_impl(dd, state, out3, workspace, static_cast<hipStream_t>(stream));
}

}  // extern "C"
