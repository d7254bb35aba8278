/*
 * dpm.h -- C ABI of the MI355X (gfx950) auxiliary-problem solver of the Difference Potentials
 * Method for the 3D Patlak-Keller-Segel system (Epshteyn & Xia, arXiv 1811.03557).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Grid: N interior nodes per axis of a cube (the set M0), spacing h, coordinate x0 of the
 *    first interior node (the same on all three axes).  Nodes on the ghost layer (N0 \ M0) carry
 *    zero Dirichlet data.  Volumes are C-ordered [z][y][x] (x fastest) over M0 only; batches are
 *    [nrhs][z][y][x].
 *  - Every pointer argument named "device" is device memory owned by the caller (for example a
 *    torch tensor); the library never frees it.  Arrays must be aligned to their element size
 *    (a view into a batch at any right-hand side is fine); workspaces to 16 bytes.
 *  - stream: a hipStream_t passed as void* (NULL = the default stream).  Work is enqueued
 *    asynchronously; results are valid after the stream is synchronised, unless the call says
 *    it synchronises.
 *  - Every call validates all of its arguments before it enqueues anything; on an error nothing
 *    is launched and dpm_last_error() returns a thread-local message.
 *  - dpm_status codes: DPM_OK success; DPM_EINVAL bad argument; DPM_ENOMEM allocation failed;
 *    DPM_EHIP a HIP runtime error; DPM_ENOTCONV iterative refinement did not reach rtol (the
 *    last iterate is in u); DPM_EGEOM invalid geometry (empty gamma or no margin to the ghost
 *    layer); DPM_ERANK the boundary least-squares matrix is rank deficient.
 */
#ifndef DPM_H
#define DPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPM_OK = 0,
  DPM_EINVAL = 1,
  DPM_ENOMEM = 2,
  DPM_EHIP = 3,
  DPM_ENOTCONV = 4,
  DPM_EGEOM = 5,
  DPM_ERANK = 6
} dpm_status;

/* Arithmetic of the per-axis sine transforms. */
typedef enum {
  DPM_FP64 = 0,   /* FP64 transforms */
  DPM_FP32 = 1,   /* FP32 transforms (FP64 residual refinement when io_fp64 and max_refine > 0) */
  DPM_BF16X3 = 2,  /* split bf16 hi/lo dense-DST on MFMA, FP32 accumulation (N <= 256) */
  DPM_FP64_GEMM = 3 /* FP64 transforms as dense DST-I products on the FP64 matrix cores (any
                       7 <= N <= 543, N + 1 need not be a power of two; FP64 I/O, no
                       refinement): the dense counterpart of DPM_FP64 */
} dpm_precision;

typedef struct {
  int32_t n;     /* interior nodes per axis, 7 <= n <= 1023; the FFT-form and split-bf16
                    transforms need n + 1 a power of two, DPM_FP64_GEMM takes any n <= 543 */
  double h;      /* mesh spacing, > 0 */
  double sigma;  /* shift of the operator sigma I - Lap_h, >= 0 and finite */
  double x0;     /* coordinate of the first interior node (geometry calls only) */
} dpm_grid;

typedef struct {
  int32_t prec;        /* dpm_precision */
  int32_t io_fp64;     /* 1: b and u are FP64; 0: FP32 (only with DPM_FP32 and max_refine == 0) */
  double rtol;         /* refinement target ||u_k - u||/||u|| (estimated), e.g. 1e-10 */
  int32_t max_refine;  /* refinement iterations after the first solve (0 = none) */
  int32_t rhs_chunk;   /* right-hand sides per batched launch (0 = library choice) */
  void* workspace;     /* device scratch of >= workspace_bytes, from dpm_workspace_size */
  size_t workspace_bytes;
  int32_t sweeps;      /* dpm_sweeps: how the FFT-form transforms pass over the volume */
} dpm_opts;

/* Sweep layout of the FFT-form solves (DPM_FP64, DPM_FP32).  A solve applies the DST-I along x
 * and y, solves the tridiagonal system along z of every spectral column (the same result as the
 * DST along z, the division by the eigenvalues and the DST back) and applies the two DST-Is
 * again; the layouts differ in how many times the volume travels through HBM.
 *  DPM_SWEEPS_AUTO (0): the library's choice: the layout dpm_autotune recorded, else
 *    DPM_SWEEPS_PLANE where available, else DPM_SWEEPS_SPLIT at n = 511 (plain solves), else
 *    DPM_SWEEPS_AXIS.
 *  DPM_SWEEPS_AXIS: five per-axis passes (x, y, z, y, x).
 *  DPM_SWEEPS_PLANE: three sweeps: both in-plane transforms of a z-plane in one pass with the
 *    plane in LDS (n = 7, 15, 31, 63, 127), the z pass, the inverse plane pass.
 *  DPM_SWEEPS_SPLIT: four passes and a small one, for plain solves (DPM_FP64 without refinement,
 *    DPM_FP32 with FP32 I/O) at n = 255 and 511: the y transforms; the x transforms of 16
 *    consecutive z-rows fused with the segment-local elimination of the z solve, and back with
 *    its reconstruction; between them the separators' reduced system, which reads 2/16 and writes
 *    1/16 of a volume.  The workspace then holds ((n + 1)/16 - 1) n^2 reals of the transform type
 *    per right-hand side of a launch (dpm_workspace_size counts them); under DPM_SWEEPS_AUTO a
 *    workspace too small for them runs the per-axis sweeps instead.
 * Results agree to rounding (the transforms and the z solve are the same, applied in another
 * order of operations).  The dense forms ignore the field. */
typedef enum {
  DPM_SWEEPS_AUTO = 0,
  DPM_SWEEPS_AXIS = 1,
  DPM_SWEEPS_PLANE = 2,
  DPM_SWEEPS_SPLIT = 3
} dpm_sweeps;

typedef struct {
  int32_t refine_iters;  /* refinement iterations actually applied (max over the batch) */
  double est_rel_err;    /* max over the batch of ||last correction||_inf / ||u||_inf */
} dpm_info;

/* Scratch bytes needed by aux_solve / aux_solve_batched for these arguments (host call). */
dpm_status dpm_workspace_size(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts,
                              size_t* bytes);

/* Right-hand sides per sweep launch that aux_solve_batched uses for nrhs right-hand sides with
 * these options (opts->rhs_chunk if set, else the library's choice for the grid size). */
dpm_status dpm_rhs_chunk(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts, int32_t* chunk);

/* Autotuner of the batched launches' shape: the number of right-hand sides a sweep launch
 * carries (the width); where a fused layout exists (FFT form: the plane sweeps at n <= 127, the
 * split layout at n = 255, 511 for plain solves), the sweep layout (dpm_sweeps); and, for the
 * FFT and Bluestein forms, the tile of the z pass (columns per block:
 * 16, 32 or 64, each thread one 16-row segment of a column).  The width sets the launch count
 * and how much of a launch's working set the 256 MB Infinity Cache holds; the layout trades two
 * fewer passes over HBM against the fused kernels' lower occupancy; the z tile trades the width
 * of a wavefront's contiguous runs against blocks per CU; so the best shape depends on n, the
 * precision and the chip.  (It suits the batched right-hand sides of the boundary-matrix build,
 * Step 2 of the paper's algorithm, and any batch of auxiliary problems.)
 *
 * Times aux_solve_batched(grid, nrhs, b, u, opts) for each candidate width in
 * {1, 2, 3, 4, 6, 8, 12, 16} that is at most nrhs, whose workspace fits
 * opts->workspace_bytes, and (for options that keep a transform workspace: FP32 with FP64 I/O,
 * refined FP64, BF16X3) at most the library's default width, so that a workspace sized before
 * tuning stays large enough; with opts->sweeps == DPM_SWEEPS_AUTO every width is timed in both
 * layouts where both exist, else in the given layout.  opts->rhs_chunk is ignored.  Each
 * candidate takes one untimed solve, then `reps` solves timed with HIP events on `stream`; the
 * fastest is kept, and ties keep the earlier candidate (narrower width, per-axis layout first).
 * Then, at the winning width and layout (unless it is the split layout, which has no z pass),
 * the z pass is timed at each column count whose
 * segments fit one block (ceil((n + 1) / 16) * columns <= 1024); one replaces the default only
 * when strictly faster than every candidate before it.
 *
 * The winning shape is recorded for (current device, n, prec, io_fp64, max_refine > 0).  From
 * then on every solve with opts->rhs_chunk == 0 uses its width, as do dpm_workspace_size and
 * dpm_rhs_chunk, every solve with opts->sweeps == DPM_SWEEPS_AUTO its layout, and every solve its
 * z tile.  A solve's results do not depend on the width or the z tile; the layouts agree to
 * rounding.
 *
 * b and u are caller-owned device arrays as for aux_solve_batched, and u is overwritten with
 * the solution.  The outputs are host arrays, each nullable: widths, sweeps, zcols and ms of
 * DPM_TUNE_MAX_CANDIDATES entries (each candidate's width, layout, z-pass columns per block --
 * 0 for the default -- and best time per batched solve, in ms), *count (candidates timed),
 * *best, *best_sweeps and *best_zcols (the shape recorded; 0: the default z tile).  The call
 * synchronises the stream.
 *
 * Errors: those of aux_solve_batched; DPM_EINVAL for reps outside [1, 100], for a workspace that
 * fits no candidate, or while sweep timing is on.  The table is process-wide and guarded by a
 * lock; a solve reads it once and takes either the old pair or the new.  A solve whose
 * workspace (opts->rhs_chunk == 0) is smaller than the recorded width needs, for example one
 * sized before a re-tune or a reset, runs at the widest width the workspace holds. */
#define DPM_TUNE_MAX_CANDIDATES 24
dpm_status dpm_autotune(const dpm_grid* grid, int32_t nrhs, const dpm_opts* opts, const void* b,
                        void* u, int32_t reps, void* stream, int32_t* widths, int32_t* sweeps,
                        int32_t* zcols, double* ms, int32_t* count, int32_t* best,
                        int32_t* best_sweeps, int32_t* best_zcols);

/* Forgets every recorded shape: solves go back to the library's default widths, layouts and z
 * tiles. */
void dpm_autotune_reset(void);

/* Builds the per-(device, n) tables (sine/twiddle and eigenvalue tables) ahead of time.  The
 * first solve of a size does this by itself; call it first when that solve is captured into a
 * HIP graph, since building uploads with synchronous copies. */
dpm_status dpm_prepare(int32_t n);

/*
 * aux_solve -- the discrete auxiliary problem (paper Sec. 2, Definition of the AP, eqs
 * discrete_ap and discrete_ap_boundary) in sigma-form:
 *     (sigma I - Lap_h) u = b on M0,  u = 0 on N0 \ M0,
 * with Lap_h the 7-point Laplacian (eq stencil:7-point).  The paper's AP with operator
 * L = I - dt Lap_h and right-hand side q is this call with sigma = 1/dt and b = q/dt.
 * b, u: device, N^3 values, FP64 when opts->io_fp64 else FP32.  b and u must not overlap.
 * info: host, nullable; when given, the call synchronises the stream to fill it.
 */
dpm_status aux_solve(const dpm_grid* grid, const void* b, void* u, const dpm_opts* opts,
                     void* stream, dpm_info* info);

/* nrhs independent auxiliary problems with the same grid and sigma: b, u are [nrhs][N^3]. */
dpm_status aux_solve_batched(const dpm_grid* grid, int32_t nrhs, const void* b, void* u,
                             const dpm_opts* opts, void* stream, dpm_info* info);

/* aux_solve_batched with one shift per right-hand side: right-hand side r is solved with
 * sigma[r] (host array of nrhs finite values >= 0; grid->sigma is ignored).  The shifts are
 * copied to the workspace on the stream before the call returns, so the host array may be
 * reused at once.  Lets requests with different time steps share one batched launch. */
dpm_status aux_solve_batched_sigma(const dpm_grid* grid, int32_t nrhs, const double* sigma,
                                   const void* b, void* u, const dpm_opts* opts, void* stream,
                                   dpm_info* info);

/* Bytes of the device scratch that aux_solve_batched_noalloc uses (64 MiB on every device the
 * library runs on, held from library load until the process ends).  Enough for one 255^3 FP32
 * transform volume plus the refinement state of up to several thousand right-hand sides. */
#define DPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* aux_solve_batched for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The call allocates nothing: it
 * takes no workspace from the caller (opts->workspace and opts->workspace_bytes are ignored)
 * and puts the refinement state and the transform volumes in a library-owned static device
 * array of DPM_NOALLOC_SCRATCH_BYTES per device.  Arguments, layouts and results are those of
 * aux_solve_batched (the same kernels); the launch width is the one aux_solve_batched would use,
 * narrowed to what the static scratch holds.
 * Errors: those of aux_solve_batched; DPM_EINVAL when even one right-hand side per launch does
 * not fit the static scratch (for example FP32 transforms at n = 511), with nrhs so large that
 * the per-right-hand-side state alone exceeds it, or when the size's tables were never built on
 * the current device (call dpm_prepare(n) once at set-up: building them allocates).
 * Every call on one device shares that device's scratch and leaves its contents behind (the
 * state that must start at zero is cleared by a kernel at the start of each call): calls that
 * overlap on one device, on different streams or threads, race and must be serialised by the
 * caller. */
dpm_status aux_solve_batched_noalloc(const dpm_grid* grid, int32_t nrhs, const void* b, void* u,
                                     const dpm_opts* opts, void* stream, dpm_info* info);

/* Geometry of the domain Omega inside the cube: a sphere (axes[0] = radius) or an ellipsoid
 * with semi-axes (axes[0], axes[1], axes[2]) along (x, y, z). */
typedef struct {
  int32_t kind;       /* 0 sphere, 1 ellipsoid */
  double center[3];   /* (x, y, z) */
  double axes[3];
} dpm_geometry;

/* M+ mask (paper Def. "point sets"): m_plus[i] = 1 if node i lies strictly inside Omega, else
 * 0.  m_plus: device, N^3 uint8. */
dpm_status dpm_classify(const dpm_grid* grid, const dpm_geometry* geom, uint8_t* m_plus,
                        void* stream);

/*
 * dpm_gamma_points -- the discrete grid boundary gamma = N+ cap N-, gamma_in = M+ cap gamma
 * (paper Def. "point sets").  Two-call pattern: with idx == NULL only the counts are returned;
 * otherwise idx (device, n_gamma int32) receives the linear indices of gamma in ascending order
 * and is_in (device, n_gamma uint8) flags gamma_in.  m_plus: device N^3 uint8.  Synchronises
 * the stream (the counts are host values).  DPM_EGEOM if gamma is empty or N+ touches the
 * ghost layer.
 */
dpm_status dpm_gamma_points(const dpm_grid* grid, const uint8_t* m_plus, int32_t* n_gamma,
                            int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, void* stream);

/*
 * dpm_basis -- spectral densities of the extension operator (paper Sec. 2, eqs
 * extension_operator1, spectral_approximation_sd, extension_operator_recast): for each gamma
 * node, its projection onto Gamma (signed distance d, positive outside; polar/azimuthal angles
 * of the foot point, parametric angles for an ellipsoid) and the real orthonormal spherical
 * harmonics Y_lm, l <= lmax, m = -l..l, without Condon-Shortley phase.  basis: device,
 * n_basis x n_gamma FP64 (row nu contiguous), n_basis = (beta + 1)(lmax + 1)^2; rows
 * (lmax+1)^2 .. carry (d^2/2) Y_lm when beta = 1.  d_out (nullable, device n_gamma FP64)
 * receives d.
 */
dpm_status dpm_basis(const dpm_grid* grid, const dpm_geometry* geom, int32_t n_gamma,
                     const int32_t* idx, int32_t lmax, int32_t beta, double* basis,
                     double* d_out, void* stream);

typedef struct dpm_bep dpm_bep; /* library-owned: mask, gamma lists, basis, BEP matrix, QR */

/*
 * dpm_basis_zonal -- zonal densities of the extension operator, the paper's basis for initial
 * data symmetric about the z axis ("Basis functions, extension operators and BEPs"; remark (i)
 * of the spectral approach): P_nu(cos theta), the unnormalised Legendre polynomials of degree
 * nu = 0..mmax of the polar angle of each gamma node's projection onto Gamma.  basis: device,
 * n_basis x n_gamma FP64 (row nu contiguous), n_basis = (beta + 1)(mmax + 1); rows mmax + 1 ..
 * carry (d^2/2) P_nu when beta = 1 (the 3-term extension), none when beta = 0 (the 2-term
 * extension with zero Neumann data).  d_out (nullable, device n_gamma FP64) receives d.
 */
dpm_status dpm_basis_zonal(const dpm_grid* grid, const dpm_geometry* geom, int32_t n_gamma,
                           const int32_t* idx, int32_t mmax, int32_t beta, double* basis,
                           double* d_out, void* stream);

/*
 * dpm_build_boundary_matrix -- paper Algorithm "Main Steps", Step 2: the reduced-BEP matrix
 * (eq BEP_recast) A[:, nu] = Tr_gamma_in (I - P_gamma) basis_nu, one AP solve per column with
 * right-hand side 1_{M-} (sigma - Lap_h)[basis_nu extended by zero] (Def. "DP" in sigma-form),
 * followed by an FP64 QR A = Q R and the least-squares operator P = R^-1 Q1^T (Q1: the first
 * n_basis columns of Q), kept in the handle.  The QR is CholeskyQR2 (two Gram/Cholesky passes);
 * when a Cholesky factor breaks down or the second pass finds the first far from orthogonal,
 * the Householder QR of the untouched A is used instead.
 * m_plus: device N^3 uint8; basis: device n_basis x n_gamma FP64 in the order of
 * dpm_gamma_points.  opts selects the precision of the solves (refinement applies).
 * A_out: nullable device |gamma_in| x n_basis FP64, column-major.  Allocates the handle's
 * device memory and synchronises the stream.  Release with dpm_bep_destroy.
 */
dpm_status dpm_build_boundary_matrix(const dpm_grid* grid, const uint8_t* m_plus,
                                     int32_t n_basis, const double* basis, const dpm_opts* opts,
                                     void* stream, dpm_bep** out, double* A_out);

/* Counts of a built handle (host values). */
dpm_status dpm_bep_info(const dpm_bep* bep, int32_t* n_gamma, int32_t* n_gamma_in,
                        int32_t* n_basis, double* min_abs_rdiag, double* max_abs_rdiag);

/* The QR behind a handle's least-squares operator, as of its last build or rebuild:
 * CholeskyQR2 where both Cholesky factors exist, the second pass finds the first close to
 * orthogonal (every |R2_ii - 1| <= 0.05) and min / max |R_ii| >= 1e-5; the Householder QR
 * otherwise; the Householder QR with the truncated pseudo-inverse of R when rcond > 0
 * (domain decomposition, Case 2).  The least-squares solution is the same; the methods differ in
 * cost (CholeskyQR2 is two Gram products and small factorisations, the Householder QR one
 * dependent launch per column) and in rounding. */
typedef enum {
  DPM_LSQ_CHOLESKY_QR2 = 1,
  DPM_LSQ_HOUSEHOLDER = 2,
  DPM_LSQ_HOUSEHOLDER_TRUNCATED = 3
} dpm_lsq_method;
dpm_status dpm_bep_lsq_method(const dpm_bep* bep, int32_t* method);

/* Device bytes the handle holds (masks, gamma lists, densities, the factored matrix, the
 * least-squares operator): what keeping it resident costs, e.g. for admission by HBM footprint. */
dpm_status dpm_bep_device_bytes(const dpm_bep* bep, size_t* bytes);

/*
 * dpm_bep_solve -- paper Step 5: least-squares coefficients C = argmin ||A C - g||_2 of the
 * reduced BEP (eq BEP_recast), as C = P g with the operator P = R^-1 Q1^T formed from the QR at
 * build time.  g: device nvec x |gamma_in| FP64; C: device nvec x n_basis FP64.  Asynchronous;
 * allocates nothing.
 */
dpm_status dpm_bep_solve(const dpm_bep* bep, int32_t nvec, const double* g, double* C,
                         void* stream);

/* Scratch bytes needed by dpm_step with these options. */
dpm_status dpm_step_workspace_size(const dpm_bep* bep, const dpm_opts* opts, size_t* bytes);

/*
 * dpm_step -- one IMEX time step of the DPM (paper Algorithm "Main Steps", Steps 4a, 5, 6, 7)
 * for both species with L = I - dt Lap_h (the handle must have been built with sigma = 1/dt):
 *   f_rho = rho - dt g (upwind, minmod; eqs discrete_convective_term .. slope_limiter),
 *   f_c = (1 - dt) c + dt rho on M+ (eq discrete_chemotaxis, alpha = gamma_rho = gamma_c = 1);
 *   particular solutions G f, Tr_gamma_in G f, coefficients by least squares, densities
 *   u_gamma = basis^T C, and the discrete generalized Green's formula u = P u_gamma + G f on
 *   N+ (computed as one AP solve per species by linearity).
 * rho_in, c_in: device N^3 FP64 values on N+ (other entries ignored); rho_out, c_out: device
 * N^3 FP64, zero off N+, two different buffers (DPM_EINVAL otherwise); they may alias the
 * inputs.  All four 8-byte aligned, opts->workspace 16-byte aligned.  chi: chemotactic
 * sensitivity.
 * info: host, nullable (synchronises when given).
 */
dpm_status dpm_step(const dpm_bep* bep, double dt, double chi, const double* rho_in,
                    const double* c_in, double* rho_out, double* c_out, const dpm_opts* opts,
                    void* stream, dpm_info* info);

/*
 * dpm_stepper -- the time loop of the paper's Algorithm "Main Steps" (Steps 4a-7 repeated) on
 * fixed buffers: dpm_stepper_create captures one dpm_step that updates (rho, c) in place into a
 * HIP graph; dpm_stepper_run replays it nsteps times on `stream`.  Each replay also checks the
 * step's outputs for non-finite values on the device; dpm_stepper_first_nonfinite returns the
 * number (from 1, counted since create) of the first step whose output held one, or 0.
 * rho, c: device N^3 FP64 state, updated in place by every replay; opts->workspace: at least
 * dpm_step_workspace_size bytes.  Both must stay valid, and must not be used by other work
 * while replays run, until dpm_stepper_destroy.  The handle keeps a pointer to bep: destroy the
 * stepper first.  create enqueues the guard's reset on `stream`; it fails with DPM_EINVAL while
 * sweep timing is enabled.  first_nonfinite synchronises `stream`; destroy synchronises the
 * device.  Replays of one stepper on different streams race.
 */
typedef struct dpm_stepper dpm_stepper;
dpm_status dpm_stepper_create(const dpm_bep* bep, double dt, double chi, double* rho, double* c,
                              const dpm_opts* opts, void* stream, dpm_stepper** out);
dpm_status dpm_stepper_run(dpm_stepper* st, int32_t nsteps, void* stream);
dpm_status dpm_stepper_first_nonfinite(const dpm_stepper* st, void* stream, int32_t* step);
void dpm_stepper_destroy(dpm_stepper* st);

/*
 * dpm_cfl_scan -- paper Algorithm "Main Steps", Steps 3 and 8: the quantities the adaptive time
 * loop decides on.  out2[0] = max |grad_h c| over the six faces of every M+ node (the face
 * differences (c_nb - c) / h of eq cfl_condition, neighbours in N+), out2[1] = max |rho| over
 * M+.  The CFL-type bound of the positivity theorem is then dt <= h / (6 chi out2[0]).  A
 * non-finite value anywhere in the scanned entries makes the corresponding output NaN.
 * rho, c: device N^3 FP64; out2: device, 2 FP64.  Asynchronous; allocates nothing.
 */
dpm_status dpm_cfl_scan(const dpm_bep* bep, const double* rho, const double* c, double* out2,
                        void* stream);

/* Scratch bytes dpm_bep_rebuild needs for this handle (host call): the right-hand sides,
 * solutions and solve workspace of one batch of column solves, or the factorisation's
 * temporaries, whichever is larger (the two phases run one after the other). */
dpm_status dpm_bep_rebuild_workspace_size(const dpm_bep* bep, size_t* bytes);

/*
 * dpm_bep_rebuild -- paper Step 4b: recompute the reduced-BEP matrix (the same densities and
 * geometry), its QR (as dpm_build_boundary_matrix) and the least-squares operator in place for a
 * new sigma (= 1/dt), with the transform options given at build time.  workspace: device
 * scratch of at least dpm_bep_rebuild_workspace_size bytes, 16-byte aligned, owned by the
 * caller; the call allocates nothing.  Synchronises `stream` twice: once inside the QR (its
 * CholeskyQR2 check) and once for the rank test.  Errors as
 * dpm_build_boundary_matrix; after a failure the handle must only be destroyed.  A stepper built
 * on this handle keeps replaying its own dt: create a new one after a rebuild.
 */
dpm_status dpm_bep_rebuild(dpm_bep* bep, double sigma, void* workspace, size_t workspace_bytes,
                           void* stream);

/* Scratch bytes dpm_run needs with these options (host call): the dpm_step workspace, 256 bytes
 * of scanned maxima, and the rebuild scratch of dpm_bep_rebuild_workspace_size. */
dpm_status dpm_run_workspace_size(const dpm_bep* bep, const dpm_opts* opts, size_t* bytes);

/*
 * dpm_run -- the adaptive time loop of the paper's Algorithm "Main Steps" (Steps 3-8) on (rho, c)
 * in place, starting at t = 0 with the dt of the handle (dt_0 = 1/sigma: Step 2 builds with the
 * largest step, 0.5 h^2 in the paper).  Each step: scan (dpm_cfl_scan); stop if max |rho| over
 * M+ exceeds rho_cap (Step 8), has grown by at least rho_jump_cap since the previous scan, or a
 * scanned value is not finite; dt = min(h / (6 chi max|grad c|),
 * dt_prev) (Step 3; dt never grows, so the matrix of the last rebuild always belongs to the
 * current dt); if dt < dt_prev rebuild the matrix at sigma = 1/dt (Step 4b); one dpm_step
 * (Steps 4a-7); t += dt.  The loop ends when t >= t_final, after max_steps steps, or at a stop.
 * One 32-byte device-to-host copy and one synchronisation per step; a rebuild adds one more
 * (the CholeskyQR2 check inside its QR), and its rank test is read back with the next step's
 * scan (on DPM_ERANK the state holds the step taken with the rank-deficient matrix).  opts->workspace: at least dpm_run_workspace_size
 * bytes; the loop allocates nothing, rebuilds included.  dt_hist and rebuilt_hist (host,
 * nullable, max_steps entries) receive each step's dt and whether it rebuilt (1/0).  On return
 * the handle holds the matrix of the last dt.
 */
typedef struct {
  double chi;       /* chemotactic sensitivity */
  double t_final;   /* final time */
  double rho_cap;   /* Step 8 threshold on max |rho| over M+ */
  int32_t max_steps;
  double rho_jump_cap;  /* stop once max |rho| over M+ has grown by at least this much in one
                           step (the paper's termination rule for Test B, Sec. 4: 1000); a value
                           <= 0 disables it */
} dpm_run_params;
typedef enum {
  DPM_RUN_TFINAL = 0, DPM_RUN_MAXSTEPS = 1, DPM_RUN_RHOCAP = 2, DPM_RUN_NONFINITE = 3,
  DPM_RUN_RHOJUMP = 4
} dpm_run_stop;
typedef struct {
  int32_t steps;     /* steps taken */
  int32_t rebuilds;  /* Step 4b rebuilds */
  int32_t stop;      /* dpm_run_stop */
  double t;          /* time reached */
  double dt;         /* dt of the last step (1/sigma of the handle) */
  double rho_max;    /* max |rho| over M+ at the last scan */
  double grad_max;   /* max |grad_h c| at the last scan */
} dpm_run_info;
dpm_status dpm_run(dpm_bep* bep, const dpm_run_params* params, double* rho, double* c,
                   const dpm_opts* opts, void* stream, dpm_run_info* info, double* dt_hist,
                   uint8_t* rebuilt_hist);

/*
 * dpm_gauss_state -- initial data amp * exp(-rate |x - center|^2) (paper Sec. 4, Tests A and B)
 * at the nodes of M+ and, on gamma, at the projection of each node onto Gamma (paper eq
 * boundary_approx); zero elsewhere.  out: device N^3 FP64.
 */
dpm_status dpm_gauss_state(const dpm_bep* bep, const dpm_geometry* geom, double amp,
                           double rate, const double center[3], double* out, void* stream);

void dpm_bep_destroy(dpm_bep* bep);

/*
 * Domain decomposition, Case 1 (paper Sec. 3: "Case 1" and "BEPs for Case 1", eqs
 * interface_condition, DD1_BEP1, DD1_BEP2, reduced_DD1_BEP1, reduced_DD1_BEP2).  Omega, the ball
 * |x - center| < r_gamma, is split by the interface sphere Z, |x - center| = r_z, into Omega_1
 * (the inner ball) and Omega_2 (the shell); each is embedded in its own cube with its own mesh
 * (grid1, grid2: n, h, x0 per subdomain; nodes exactly on Z belong to neither M+).  zeta_1 is
 * Omega_1's discrete grid boundary; Omega_2's is the union of gamma near Gamma and zeta_2 near Z,
 * split at |x - center| = r_split.  Densities (zonal, P_nu(cos theta) of the polar angle about
 * center): near Gamma P_nu and, when beta = 1, (d^2/2) P_nu with d = |x - center| - r_gamma
 * (nu <= m_gamma); near Z P_nu, d P_nu and (d^2/2) P_nu with d = |x - center| - r_z (nu <= m_z),
 * the same coefficients on both sides of Z, which imposes the continuity of u and of its first
 * two normal derivatives.  Columns: [Gamma part, (beta + 1)(m_gamma + 1) ; Z part,
 * 3 (m_z + 1)].  The two reduced BEPs are solved together as one least-squares problem,
 * rows [zeta_1,in ; gamma_in of Omega_2], with the FP64 QR of the single domain.
 */
typedef struct dpm_dd dpm_dd; /* library-owned: both subdomains' point sets, densities, QR */
typedef struct {
  dpm_grid grid1;     /* mesh of Omega_1's cube; sigma = 1/dt, the same in grid2 */
  dpm_grid grid2;     /* mesh of Omega_2's cube */
  double center[3];   /* (x, y, z) */
  double r_z;         /* radius of the interface Z, 0 < r_z < r_split < r_gamma */
  double r_gamma;     /* radius of Gamma */
  double r_split;     /* gamma nodes of Omega_2 with |x - center| > r_split take the Gamma part */
  int32_t m_gamma;    /* highest degree on Gamma, >= 0 */
  int32_t beta;       /* 1: 3-term extension on Gamma, 0: 2-term (zero Neumann data both) */
  int32_t m_z;        /* highest degree on Z, >= 0 */
} dpm_dd_params;

/*
 * dpm_dd_build -- Step 2 of the paper's algorithm for both subdomains: point sets, densities,
 * one AP solve per density on each mesh, the stacked matrix [[0, A_1], [A_2]] (A_1 carries the
 * Z columns only) and its QR and least-squares operator.  opts selects the precision of the
 * solves (both grids must suit it).  A_out: nullable device rows x n_cols FP64 (rows =
 * |zeta_1,in| + |gamma_2,in|, see dpm_dd_info), column-major, the matrix before factorisation.  Allocates the handle's device
 * memory and synchronises the stream.  DPM_EGEOM when a subdomain's N+ leaves its cube,
 * DPM_ERANK when the stacked matrix is rank deficient.  Release with dpm_dd_destroy.
 */
dpm_status dpm_dd_build(const dpm_dd_params* params, const dpm_opts* opts, void* stream,
                        dpm_dd** out, double* A_out);

/*
 * dpm_dd2_build -- the same for Case 2 (paper Sec. 3: "Case 2" and "BEPs for Case 2", eqs
 * DD2_BEP and reduced_DD2_BEP, and the remark on effective densities): Omega is the ball
 * |x| < r_gamma about the origin, Z the sphere of radius r_z about q = (0, 0, q_z) with q_z - r_z
 * < r_gamma < q_z + r_z, so Z meets Gamma on a circle (polar angle theta* about the origin,
 * angle psi* at q from the direction towards the origin); Omega_1 = Omega cap {|x - q| < r_z},
 * Omega_2 = Omega cap {|x - q| > r_z}.  On subdomain l's mesh, gamma_l = the nodes of the ball's
 * discrete grid boundary whose polar angle is at most theta* + eps (l = 1) or at least
 * theta* - eps (l = 2), zeta_l = the nodes of the discrete grid boundary of Z's side whose angle
 * psi is at most psi* + eps_z, with eps = eps_layers h_l / r_gamma and eps_z = eps_layers h_l /
 * r_z.  Densities: one zonal expansion on Gamma (P_nu(cos theta) and, beta = 1, (d^2/2) P_nu,
 * nu <= m_gamma) shared by gamma_1 and gamma_2, one 3-term expansion on Z (P_nu(cos psi), d P_nu,
 * (d^2/2) P_nu, nu <= m_z) shared by zeta_1 and zeta_2.  A node in gamma_l and zeta_l carries
 * the average of its two densities in the difference potential and two reduced-BEP equations
 * (Gamma row first).  Rows follow each subdomain's gamma_in in ascending index, subdomain 1 first.
 * Node coordinates of mesh l are (x0 + h i) + origin_l per axis.  DPM_EGEOM also when a node of
 * a subdomain's discrete grid boundary falls in neither part (eps_layers too small).  The handle
 * is used with dpm_dd_info, dpm_dd_masks, dpm_dd_step, dpm_dd_gauss_state and dpm_dd_destroy.
 */
typedef struct {
  dpm_grid grid1;      /* mesh of Omega_1's cube; sigma = 1/dt, the same in grid2 */
  dpm_grid grid2;      /* mesh of Omega_2's cube */
  double origin1[3];   /* (x, y, z) offset of mesh 1's node coordinates */
  double origin2[3];
  double r_gamma;      /* radius of Gamma */
  double q_z;          /* centre of Z on the z axis */
  double r_z;          /* radius of Z */
  double eps_layers;   /* angular tolerance of the parts, in mesh widths, > 0 */
  int32_t m_gamma;     /* highest degree on Gamma, >= 0 */
  int32_t beta;        /* 1: 3-term extension on Gamma, 0: 2-term */
  int32_t m_z;         /* highest degree on Z, >= 0 */
  double rcond;        /* least squares of the coupled BEPs: 0 = plain (full column rank
                          required: DPM_ERANK otherwise); 0 < rcond < 1 = minimum-norm solution
                          with the singular values <= rcond * s_max taken as zero (for the
                          numerically rank-deficient matrices of many harmonics on Z's arc; at
                          most 640 columns) */
} dpm_dd2_params;
dpm_status dpm_dd2_build(const dpm_dd2_params* params, const dpm_opts* opts, void* stream,
                         dpm_dd** out, double* A_out);

/* Counts of a built handle (host values; arrays of two entries, subdomain 1 first): gamma and
 * gamma_in sizes, reduced-BEP rows (gamma_in, plus the wedge nodes' second rows in Case 2). */
dpm_status dpm_dd_info(const dpm_dd* dd, int32_t n_gamma[2], int32_t n_gamma_in[2],
                       int32_t n_rows[2], int32_t* n_cols, double* min_abs_rdiag,
                       double* max_abs_rdiag);

/* Least squares of a built handle (host values, each nullable): the rcond it was built with,
 * the numerical rank of the coupled matrix (its column count when rcond = 0) and the smallest
 * kept singular value over the largest (0 when rcond = 0).  Refreshed by every rebuild. */
dpm_status dpm_dd_lsq_info(const dpm_dd* dd, double* rcond, int32_t* rank, double* smin_ratio);
/* The QR of the coupled least squares (dpm_lsq_method; see dpm_bep_lsq_method). */
dpm_status dpm_dd_lsq_method(const dpm_dd* dd, int32_t* method);

/* Copies of subdomain l's (0 or 1) M+ and N+ masks (device, its N^3 uint8; each nullable). */
dpm_status dpm_dd_masks(const dpm_dd* dd, int32_t l, uint8_t* m_plus, uint8_t* n_plus,
                        void* stream);

/* Scratch bytes needed by dpm_dd_step with these options. */
dpm_status dpm_dd_step_workspace_size(const dpm_dd* dd, const dpm_opts* opts, size_t* bytes);

/*
 * dpm_dd_step -- one IMEX time step on both subdomains (paper Algorithm "Main Steps", Steps
 * 4a-7, with the coupled BEP of Case 1 in Step 5): forcing and particular solutions on each mesh,
 * coefficients from the stacked traces by one least squares, each subdomain's densities and its
 * discrete generalized Green's formula.  The handle must have been built with sigma = 1/dt.
 * in = {rho_1, c_1, rho_2, c_2}: device FP64 volumes of the subdomains' meshes (values on N+
 * used); out: the same four, zero off N+, four different buffers (each may alias its own
 * input).  opts->workspace: at least
 * dpm_dd_step_workspace_size bytes.  Asynchronous; allocates nothing.  Omega_2's share runs on a
 * stream owned by the handle, forked from `stream` and joined back to it by events, so the two
 * meshes' solves overlap; work enqueued on `stream` afterwards sees all four outputs.  Calls on
 * one handle must not overlap (they share that stream's events).
 */
dpm_status dpm_dd_step(const dpm_dd* dd, double dt, double chi, const double* const in[4],
                       double* const out[4], const dpm_opts* opts, void* stream);

/* amp exp(-rate |x - c0|^2) at the nodes of subdomain l's N+, zero elsewhere: the initial data
 * of the paper's Tests A and B on one mesh.  out: device FP64 volume of that mesh. */
dpm_status dpm_dd_gauss_state(const dpm_dd* dd, int32_t l, double amp, double rate,
                              const double c0[3], double* out, void* stream);

/*
 * dpm_dd_stepper -- the fixed-dt time loop on the decomposed domain: dpm_dd_stepper_create
 * captures one dpm_dd_step that updates state = {rho_1, c_1, rho_2, c_2} in place (both meshes'
 * kernels, the side stream's branch included) into a HIP graph; dpm_dd_stepper_run replays it
 * nsteps times on `stream`.  state and opts->workspace (at least dpm_dd_step_workspace_size
 * bytes) must stay valid and unused by other work while replays run, until
 * dpm_dd_stepper_destroy (which synchronises the device).  The stepper keeps pointers into the
 * handle: destroy it first; a rebuild of the handle needs a new stepper.
 */
typedef struct dpm_dd_stepper dpm_dd_stepper;
dpm_status dpm_dd_stepper_create(const dpm_dd* dd, double dt, double chi, double* const state[4],
                                 const dpm_opts* opts, dpm_dd_stepper** out);
dpm_status dpm_dd_stepper_run(dpm_dd_stepper* st, int32_t nsteps, void* stream);
void dpm_dd_stepper_destroy(dpm_dd_stepper* st);

/* Scratch bytes dpm_dd_rebuild needs (host call): the larger of either subdomain's column
 * scratch and the stacked factorisation's temporaries, plus 256 bytes. */
dpm_status dpm_dd_rebuild_workspace_size(const dpm_dd* dd, size_t* bytes);

/*
 * dpm_dd_rebuild -- Step 4b on the decomposed domain: both subdomains' columns, the stacked
 * matrix, its QR and least-squares operator again at a new sigma (= 1/dt), in place.
 * workspace: device scratch of at least dpm_dd_rebuild_workspace_size bytes, 16-byte aligned;
 * the call allocates nothing.  Synchronises `stream` twice (the CholeskyQR2 check of the plain
 * least squares, then the rank test; rcond > 0 only the second).  After a failure the handle
 * must only be destroyed.
 */
dpm_status dpm_dd_rebuild(dpm_dd* dd, double sigma, void* workspace, size_t workspace_bytes,
                          void* stream);

/* Scratch bytes dpm_dd_run needs with these options (host call): the dpm_dd_step workspace,
 * 256 bytes of scanned maxima and the dpm_dd_rebuild scratch. */
dpm_status dpm_dd_run_workspace_size(const dpm_dd* dd, const dpm_opts* opts, size_t* bytes);

/*
 * dpm_dd_run -- the adaptive time loop (paper Algorithm "Main Steps", Steps 3-8) on the
 * decomposed domain, state = {rho_1, c_1, rho_2, c_2} in place, from t = 0 with the handle's dt
 * (1/sigma).  Each step: scan both subdomains (max |grad_h c_l| over M+_l, max |rho_l| over
 * M+_l, as dpm_cfl_scan); stop if a scanned value is not finite or max |rho| over both exceeds
 * rho_cap; dt = min(dt_prev, h_l / (6 chi max|grad_h c_l|) for l = 1, 2) (each subdomain's
 * CFL-type bound on its own mesh); if dt < dt_prev dpm_dd_rebuild at 1/dt; one dpm_dd_step.
 * Ends as dpm_run (a rebuild's rank test is read back with the next scan).  opts->workspace: at
 * least dpm_dd_run_workspace_size bytes; the loop allocates nothing, rebuilds included.  info,
 * dt_hist, rebuilt_hist as for dpm_run (grad_max and rho_max: the larger of the two subdomains).
 */
dpm_status dpm_dd_run(dpm_dd* dd, const dpm_run_params* params, double* const state[4],
                      const dpm_opts* opts, void* stream, dpm_run_info* info, double* dt_hist,
                      uint8_t* rebuilt_hist);

void dpm_dd_destroy(dpm_dd* dd);

/*
 * Run diagnostics (paper Sec. 4, "Error metrics and quantities of interest", eqs sd-norm:max,
 * sd-norm:second-moment, sd-norm:free-energy and their DD forms): out3[0] = max |rho| over M+,
 * out3[1] = sum over M+ of h^3 |x|^2 rho (x the node coordinates), out3[2] = the free energy
 * sum over M+ of h^3 (rho ln rho - rho c + c^2/2 + (1/(8 h^2)) sum over the axes of
 * (c_{+1} - c_{-1})^2), with rho ln rho = 0 for rho <= 0 (rounding-level negatives; a NaN rho
 * makes the free energy and the maximum NaN).  The decomposed
 * form takes the maximum over both subdomains and adds their sums, each with its own h.
 * rho, c (state): device FP64 volumes; out3: device, 3 FP64; workspace: device scratch of at least
 * DPM_DIAG_WORKSPACE_BYTES.  Deterministic (fixed reduction order); asynchronous; allocates
 * nothing.
 */
#define DPM_DIAG_WORKSPACE_BYTES ((size_t)24576)
dpm_status dpm_diagnostics(const dpm_bep* bep, const double* rho, const double* c, double* out3,
                           void* workspace, size_t workspace_bytes, void* stream);
dpm_status dpm_dd_diagnostics(const dpm_dd* dd, const double* const state[4], double* out3,
                              void* workspace, size_t workspace_bytes, void* stream);

/*
 * Measurement support (not part of the method): while enabled, the sweep kernels launched for a
 * sampled chunk of right-hand sides are bracketed by hipEvents on the stream they run on.  A
 * chunk [rhs0, rhs0 + nb) of a solve call is sampled when it holds an index that is a multiple of
 * rhs_stride (1 = every launch; a larger stride keeps the events' own cost out of the timed
 * work).  dpm_timing_end synchronises the events and returns, per sweep kind, the number of timed
 * launches and their mean duration in ms.  Kinds: 0 first x sweep, 1 y sweep, 2 z pass,
 * 3 last x sweep, 4 residual x sweep, 5 update x sweep, 6 forward plane sweep (any input kind),
 * 7 inverse plane sweep (any output kind), 8 x sweep with the z elimination, 9 separator pass,
 * 10 x sweep with the z reconstruction (the last three: split layout, whose y sweeps count as
 * kind 1).  At most max_launches launches are
 * recorded.  Process-wide, not thread safe.
 */
dpm_status dpm_timing_begin(int32_t max_launches, int32_t rhs_stride);
dpm_status dpm_timing_end(int32_t nkinds, int32_t* counts, double* mean_ms);

/* Thread-local text of the last error (empty string when none). */
const char* dpm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DPM_H */
