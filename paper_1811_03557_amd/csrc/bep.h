// Internal layout of the boundary-equation handle and the helpers shared by the DPM kernels.
#pragma once

#include "common.h"

struct dpm_bep {
  dpm_grid grid{};
  dpm_opts opts{};          // precision of the AP solves (workspace fields unused)
  int n_gamma = 0, n_in = 0, n_basis = 0;
  uint8_t* m_plus = nullptr;  // N^3, 1 on M+
  uint8_t* n_plus = nullptr;  // N^3, 1 on N+ = M+ and gamma_ex
  int32_t* idx = nullptr;     // gamma, ascending linear index
  uint8_t* is_in = nullptr;   // gamma_in flags
  int32_t* idx_in = nullptr;  // linear indices of gamma_in (rows of A)
  int32_t* pos_in = nullptr;  // position of each gamma_in node inside the gamma list
  int32_t* in_zoff = nullptr; // n + 1: first gamma_in row of each z-plane (idx_in ascends)
  double* basis = nullptr;    // n_basis x n_gamma densities (row nu contiguous)
  double* A = nullptr;        // n_in x n_basis, column-major: Q^T, or Householder vectors below R
  double* tau = nullptr;      // n_basis reflector scalars
  double* P = nullptr;        // n_basis x n_in least-squares operator R^-1 Q1^T (row nu contiguous)
  int32_t* gpos = nullptr;    // N^3: position of each node in the gamma list, -1 off gamma
  double rdiag_min = 0.0, rdiag_max = 0.0;
  int lsq_method = 0;         // dpm_lsq_method of the last factorisation
};

// A captured time step (dpm_step in place on fixed buffers) replayed as a HIP graph.
struct dpm_stepper {
  const dpm_bep* bep = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int* guard = nullptr;  // inside the caller's workspace: step counter, first non-finite step
  long long steps_run = 0;
};

namespace dpm {

void fill_zero(double* p, long long n, hipStream_t s);
// out[c] = (sigma - Lap_h)[dens[c0 + c] on gamma, extended by zero] at the M- nodes where it can
// be nonzero (gamma_ex and their M- neighbours); other entries of out are left as they are.
void minus_rhs(const dpm_bep* b, const double* dens, int c0, int ncol, double* out, hipStream_t s);
// C[r] = R^-1 Q1^T g[r], r < nvec, as one product with the precomputed operator P
void qr_solve(const dpm_bep* bep, int nvec, const double* g, double* C, hipStream_t s);
// C = P Tr_gamma_in vol for nvec volumes (the traces gathered on the fly)
void qr_solve_traces(const dpm_bep* bep, int nvec, const double* vol, long long vsz, double* C,
                     hipStream_t s);

// factor = false stops after the columns (b->A unfactored, b->P unset): the handle then serves
// as one subdomain of a coupled problem that factors the stacked matrix itself.
// Step kernels on one handle's grid and point sets (the coupled subdomain step reuses them):
// b2 = sigma 1_{M+} (f_rho, f_c); u_gamma of both species from coefficient rows C, C + ldc;
// (o0, o1) = the two volumes of U restricted to N+.
void launch_pks_rhs(const dpm_bep* b, const double* rho, const double* c, double dt, double chi,
                    double* b2, hipStream_t s);
void launch_density(const dpm_bep* b, const double* C, int ldc, double* ug, hipStream_t s);
void launch_restrict(const dpm_bep* b, const double* U, double* o0, double* o1, hipStream_t s);

dpm_status build_bep_impl(const dpm_grid& g, const uint8_t* m_plus, int n_basis,
                          const double* basis, const dpm_opts& o, hipStream_t s, dpm_bep** out,
                          double* A_out, bool factor = true);
// Build scratch (device memory of the caller or of the build): the column solves' right-hand
// sides, solutions and solve workspace, and the factorisation's temporaries.  The two phases run
// one after the other on a stream, so a rebuild needs the larger of the two.
size_t columns_scratch_bytes(const dpm_bep* b);
size_t factor_scratch_bytes(int m, int n);
size_t rebuild_scratch_bytes(const dpm_bep* b);
// Columns of b->A at b->grid.sigma; enqueue only (no allocation, no synchronisation).
dpm_status bep_columns(dpm_bep* b, hipStream_t s, void* scratch, size_t bytes);
// QR of A (m x n column-major, in place), P = R^-1 Q1^T (n x m) and the device pair
// rd2 = (min, max) |R_ii|.  rcond = 0: CholeskyQR2 (one stream synchronisation), falling back to
// the Householder QR when it breaks down or A is too ill-conditioned for it; rcond > 0 always
// takes the Householder QR (enqueue only).  rcond > 0: P = R+ Q1^T with R+ the pseudo-inverse of R
// truncated at rcond (singular values <= rcond s_max dropped: the minimum-norm least-squares
// operator), and rd2[2], rd2[3] = numerical rank and smallest kept s / s_max (rd2 holds 4 values).
// method (nullable): the dpm_lsq_method used.
dpm_status lsq_factor(double* A, int m, int n, double* tau, double* P, hipStream_t s,
                      void* scratch, size_t bytes, double* rd2, double rcond = 0.0,
                      int* method = nullptr);

// Row chunks of the Gram products of an m x n matrix (partials n x n per chunk).
int gram_chunks(int m, int n);

// CholeskyQR2 scratch (cqr.hip): partial and reduced Gram matrices, the two Cholesky factors,
// their inverses and R^-1 (n x n row-major each), two breakdown counters and two check values.
struct CqrScratch {
  double *Gp, *G, *R1, *R2, *Ri1, *Ri2, *Ri, *q;
  int* bad;
};
// P = R^-1 Q^T from CholeskyQR2 of A (m x n column-major); A's buffer ends up holding Q^T
// (n x m row-major) and rd2[0..1] the (min, max) |R_ii|.  Synchronises the stream once, after
// the second Cholesky: when either factorisation broke down or pass 2 finds pass 1's Q1 far
// from orthogonal, *used = false, A is untouched and P holds scratch values (the caller then
// factors A by Householder QR).
dpm_status cqr2_operator(double* A, int m, int n, double* P, const CqrScratch& w, double* rd2,
                         hipStream_t s, bool* used);

// One-sided Jacobi SVD of the n x n triangle R of a factored A and its truncated pseudo-inverse
// Rp (n x n row-major), with W, V (np x np column-major), inv (n) and flags (2) as scratch
// (lsq_svd.hip).  The column count is padded to np, a multiple of 2 bs.
struct SvdShape {
  int bs, np, nb;
  bool ok;
};
SvdShape svd_shape(int n);
dpm_status pinv_of_r(const double* A, int m, int n, double rcond, double* Rp, double* W,
                     double* V, double* inv, unsigned long long* flags, double* rd,
                     hipStream_t s);
// K = Rp Wy for general (not triangular) n x n Rp.
void kmat_full(const double* Rp, const double* Wy, int n, double* K, hipStream_t s);
// Columns, QR and P of a single-domain handle, enqueue only (rd2 as above).
dpm_status factor_bep_enqueue(dpm_bep* b, hipStream_t s, double* A_out, void* scratch,
                              size_t bytes, double* rd2);
// DPM_ERANK unless min |R_ii| > 1e-12 max |R_ii| (NaN fails).
dpm_status rank_check(double mn, double mx);
// C[r] = P g[r] for nvec vectors g (m entries each), C rows of n entries
void lsq_apply(const double* P, int m, int n, int nvec, const double* g, double* C,
               hipStream_t s);
// Step 4b in place with caller scratch (rebuild_scratch_bytes); one synchronisation.
dpm_status rebuild_bep_impl(dpm_bep* b, double sigma, hipStream_t s, void* scratch, size_t bytes);
// Bytes dpm_run needs: the step workspace, the scan area and the rebuild scratch.
dpm_status run_workspace_impl(const dpm_bep* b, const dpm_opts& o, size_t* bytes);
dpm_status cfl_scan_impl(const dpm_bep* b, const double* rho, const double* c, double* out2,
                         hipStream_t s);
dpm_status run_impl(dpm_bep* b, const dpm_run_params& p, double* rho, double* c,
                    const dpm_opts& o, hipStream_t s, dpm_run_info* info, double* dt_hist,
                    uint8_t* rebuilt_hist);
void destroy_bep(dpm_bep* b);

}  // namespace dpm
