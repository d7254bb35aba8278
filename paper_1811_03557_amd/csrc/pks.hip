// One IMEX time step of the DPM for the chemotaxis system (paper Sec. 2, Algorithm "Main Steps",
// Steps 4a, 5, 6, 7) on the device, and the Gaussian initial data of the paper's Tests A/B.
//
//   f_rho = rho - dt g, f_c = (1 - dt) c + dt rho on M+  (eqs discrete_chemotaxis,
//     discrete_convective_term, c-central-difference, upwind_approximation,
//     truncated_taylor_expansion, slope_limiter; alpha = gamma_rho = gamma_c = 1)
//   G f = AP(sigma 1_{M+} f)  (two right-hand sides, one batched solve)
//   C = least squares of the reduced BEP against Tr_gamma_in G f (QR kept in the handle)
//   u_gamma = basis^T C
//   u = P_{N+gamma} u_gamma + G f = AP(1_{M+} sigma f + 1_{M-} (sigma - Lap_h)[u_gamma])
//     (Green's formula as one solve, by linearity of the AP), restricted to N+.
// Readings: the limited slope is zero at gamma_ex nodes; a face gradient of exactly 0 takes the
// right (downstream-cell) state, as the scheme is written.
#include <climits>
#include <cmath>

#include "bep.h"
#include "geom_dev.h"

namespace dpm {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

// b2[0] = sigma 1_{M+} f_rho, b2[1] = sigma 1_{M+} f_c.  With a stepper guard, the first
// thread also advances the step number (guard[0]) that the step's restriction records.
__global__ void k_pks_rhs(const double* __restrict__ rho, const double* __restrict__ c,
                          const uint8_t* __restrict__ mp, int n, double h, double dt, double chi,
                          double sigma, double* __restrict__ b2, int* __restrict__ guard) {
  const long long vsz = (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (guard != nullptr && i == 0) guard[0] += 1;
  if (i >= vsz) return;
  if (!mp[i]) {
    b2[i] = 0.0;
    b2[vsz + i] = 0.0;
    return;
  }
  const double r0 = rho[i], c0 = c[i];
  const double ih = 1.0 / h, hh = 0.5 * h;
  const long long st[3] = {(long long)n * n, (long long)n, 1};  // z, y, x
  double g = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const long long s = st[a];
    const double rp = rho[i + s], rm = rho[i - s];
    const double cp = c[i + s], cm = c[i - s];
    const double s0 = minmod3(2.0 * (rp - r0) * ih, (rp - rm) * (0.5 * ih), 2.0 * (r0 - rm) * ih);
    double sp = 0.0, sm = 0.0;
    if (mp[i + s]) {
      const double rpp = rho[i + 2 * s];
      sp = minmod3(2.0 * (rpp - rp) * ih, (rpp - r0) * (0.5 * ih), 2.0 * (rp - r0) * ih);
    }
    if (mp[i - s]) {
      const double rmm = rho[i - 2 * s];
      sm = minmod3(2.0 * (r0 - rm) * ih, (r0 - rmm) * (0.5 * ih), 2.0 * (rm - rmm) * ih);
    }
    const double gp = (cp - c0) * ih;  // face i + 1/2
    const double gm = (c0 - cm) * ih;  // face i - 1/2
    const double fp = chi * (gp > 0.0 ? r0 + hh * s0 : rp - hh * sp) * gp;
    const double fm = chi * (gm > 0.0 ? rm + hh * sm : r0 - hh * s0) * gm;
    g += (fp - fm) * ih;
  }
  b2[i] = sigma * (r0 - dt * g);
  b2[vsz + i] = sigma * ((1.0 - dt) * c0 + dt * r0);
}

// u_gamma[r][i] = sum_nu basis[nu][i] C[r ldc + nu] for the two species r = 0, 1: one thread per
// gamma node reads its basis column once, kDU densities in flight at a time.
constexpr int kDU = 10;
__global__ void k_density(const double* __restrict__ basis, const double* __restrict__ C,
                          int nb, int ldc, int ng, double* __restrict__ ug) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  double a0 = 0.0, a1 = 0.0;
  int nu = 0;
  for (; nu + kDU <= nb; nu += kDU) {
    double v[kDU];
#pragma unroll
    for (int u = 0; u < kDU; ++u) v[u] = basis[(long long)(nu + u) * ng + i];
#pragma unroll
    for (int u = 0; u < kDU; ++u) {
      a0 += v[u] * C[nu + u];
      a1 += v[u] * C[ldc + nu + u];
    }
  }
  for (; nu < nb; ++nu) {
    const double v = basis[(long long)nu * ng + i];
    a0 += v * C[nu];
    a1 += v * C[ldc + nu];
  }
  ug[i] = a0;
  ug[(long long)ng + i] = a1;
}

// Restriction to N+; with a guard, a non-finite output records the current step number
// (guard[0]) into guard[1] by atomic minimum: one atomic per block that holds one, skipped once
// the step is recorded (a state that is non-finite everywhere would otherwise serialise
// thousands of atomics on one address).
__global__ void k_restrict(const double* __restrict__ U, const uint8_t* __restrict__ np,
                           long long vsz, double* __restrict__ o0, double* __restrict__ o1,
                           int* __restrict__ guard) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < vsz) {
    const bool in = np[i] != 0;
    const double v0 = in ? U[i] : 0.0, v1 = in ? U[vsz + i] : 0.0;
    o0[i] = v0;
    o1[i] = v1;
    bad = !(isfinite(v0) && isfinite(v1));
  }
  if (guard == nullptr) return;
  if (__syncthreads_or(bad) && threadIdx.x == 0) {
    const int step = guard[0];
    if (guard[1] > step) atomicMin(&guard[1], step);
  }
}

// guard[0] = step number (steps count from 1: each step's forcing kernel advances it first),
// guard[1] = first step with a non-finite output
__global__ void k_guard_init(int* guard) {
  if (threadIdx.x == 0) {
    guard[0] = 0;
    guard[1] = INT_MAX;
  }
}

// amp exp(-rate |x - x_c|^2) at M+ nodes; phase 1 overwrites gamma nodes with the value at
// their projection onto Gamma
__global__ void k_gauss_nodes(const uint8_t* __restrict__ mp, int n, double h, double x0,
                              double amp, double rate, double xc, double yc, double zc,
                              double* __restrict__ out) {
  const long long vsz = (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vsz) return;
  if (!mp[i]) { out[i] = 0.0; return; }
  const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
  const double dx = x0 + h * x - xc, dy = x0 + h * y - yc, dz = x0 + h * z - zc;
  out[i] = amp * exp(-rate * (dx * dx + dy * dy + dz * dz));
}

__global__ void k_gauss_gamma(const int32_t* __restrict__ idx, int ng, int n, double h, double x0,
                              GeoDev geo, double amp, double rate, double xc, double yc,
                              double zc, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ng) return;
  const long long i = idx[k];
  const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
  double d, th, ph, q[3];
  project(geo, x0 + h * x - geo.cx, x0 + h * y - geo.cy, x0 + h * z - geo.cz, &d, &th, &ph, q);
  const double dx = geo.cx + q[0] - xc, dy = geo.cy + q[1] - yc, dz = geo.cz + q[2] - zc;
  out[i] = amp * exp(-rate * (dx * dx + dy * dy + dz * dz));
}

// Maxima of non-negative doubles as atomic maxima of their bit patterns: non-negative doubles
// order as unsigned integers, and a NaN (its sign cleared by fabs) orders above +inf, so any NaN
// in the scanned entries makes the result NaN.  Order-independent, hence deterministic.
__device__ __forceinline__ unsigned long long mag_bits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

__global__ void k_scan_init(unsigned long long* __restrict__ out2) {
  if (threadIdx.x < 2) out2[threadIdx.x] = 0ull;
}

// out2[0] = max over M+ nodes and their six faces of |c_nb - c| / h (eq cfl_condition),
// out2[1] = max over M+ of |rho|.  M+ nodes are interior to the cube, so every neighbour exists.
// A fixed grid strides over the nodes; each block reduces its maxima (waves, then LDS) and
// issues one atomic per output.
constexpr int kScanBlocks = 512;
__global__ __launch_bounds__(256) void k_cfl_scan(const double* __restrict__ rho,
                                                  const double* __restrict__ c,
                                                  const uint8_t* __restrict__ mp, int n, double h,
                                                  unsigned long long* __restrict__ out2) {
  __shared__ unsigned long long sg[4], sr[4];
  const long long vsz = (long long)n * n * n;
  const long long st[3] = {(long long)n * n, (long long)n, 1};
  unsigned long long gb = 0ull, rb = 0ull;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vsz;
       i += (long long)gridDim.x * blockDim.x) {
    if (!mp[i]) continue;
    const double c0 = c[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const unsigned long long up = mag_bits((c[i + st[a]] - c0) / h);
      const unsigned long long dn = mag_bits((c[i - st[a]] - c0) / h);
      gb = up > gb ? up : gb;
      gb = dn > gb ? dn : gb;
    }
    const unsigned long long r = mag_bits(rho[i]);
    rb = r > rb ? r : rb;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long go = __shfl_xor(gb, off), ro = __shfl_xor(rb, off);
    gb = go > gb ? go : gb;
    rb = ro > rb ? ro : rb;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sg[w] = gb; sr[w] = rb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      gb = sg[k] > gb ? sg[k] : gb;
      rb = sr[k] > rb ? sr[k] : rb;
    }
    if (gb) atomicMax(&out2[0], gb);
    if (rb) atomicMax(&out2[1], rb);
  }
}

unsigned grid1(long long n) { return (unsigned)((n + kB - 1) / kB); }

struct StepLayout {
  size_t b2, X, C, ug, guard, tr, solve_ws, total;
};

StepLayout step_layout(const dpm_bep* b, size_t solve_ws) {
  const size_t V = (size_t)b->grid.n * b->grid.n * b->grid.n * sizeof(double);
  StepLayout L;
  size_t o = 0;
  L.b2 = o; o = align_up(o + 2 * V, 256);
  L.X = o; o = align_up(o + 2 * V, 256);
  L.C = o; o = align_up(o + 2 * sizeof(double) * b->n_basis, 256);
  L.ug = o; o = align_up(o + 2 * sizeof(double) * b->n_gamma, 256);
  L.guard = o; o = align_up(o + 2 * sizeof(int), 256);
  L.tr = o; o = align_up(o + 2 * sizeof(double) * b->n_in, 256);
  L.solve_ws = o; o = align_up(o + solve_ws, 256);
  L.total = o;
  return L;
}

}  // namespace

void launch_pks_rhs(const dpm_bep* b, const double* rho, const double* c, double dt, double chi,
                    double* b2, hipStream_t s) {
  const dpm_grid& g = b->grid;
  const long long vsz = (long long)g.n * g.n * g.n;
  hipLaunchKernelGGL(k_pks_rhs, dim3(grid1(vsz)), dim3(kB), 0, s, rho, c, b->m_plus, g.n, g.h,
                     dt, chi, g.sigma, b2, nullptr);
}

void launch_density(const dpm_bep* b, const double* C, int ldc, double* ug, hipStream_t s) {
  hipLaunchKernelGGL(k_density, dim3(grid1(b->n_gamma)), dim3(kB), 0, s, b->basis, C,
                     b->n_basis, ldc, b->n_gamma, ug);
}

void launch_restrict(const dpm_bep* b, const double* U, double* o0, double* o1, hipStream_t s) {
  const long long vsz = (long long)b->grid.n * b->grid.n * b->grid.n;
  hipLaunchKernelGGL(k_restrict, dim3(grid1(vsz)), dim3(kB), 0, s, U, b->n_plus, vsz, o0, o1,
                     nullptr);
}

dpm_status step_workspace_impl(const dpm_bep* b, const dpm_opts& o, size_t* bytes) {
  size_t sw = 0;
  dpm_opts so = o;
  so.rhs_chunk = 2;  // both species in one launch: the size never depends on tuning
  DPM_TRY(workspace_size_impl(b->grid, 2, so, &sw));
  *bytes = step_layout(b, sw).total;
  return DPM_OK;
}

namespace {

// Steps 4a-7 enqueued on s; no host synchronisation, so the sequence can be captured.
dpm_status step_enqueue(const dpm_bep* b, double dt, double chi, const double* rho_in,
                        const double* c_in, double* rho_out, double* c_out, const dpm_opts& o,
                        hipStream_t s, dpm_info* info, bool guard) {
  const dpm_grid& g = b->grid;
  size_t sw = 0;
  dpm_opts so = o;
  so.rhs_chunk = 2;  // both species in one launch: the size never depends on tuning
  DPM_TRY(workspace_size_impl(g, 2, so, &sw));
  const StepLayout L = step_layout(b, sw);
  if (o.workspace == nullptr || o.workspace_bytes < L.total) {
    set_error("dpm_step: workspace too small: %zu bytes given, %zu needed", o.workspace_bytes, L.total);
    return DPM_EINVAL;
  }
  char* ws = static_cast<char*>(o.workspace);
  double* b2 = reinterpret_cast<double*>(ws + L.b2);
  double* X = reinterpret_cast<double*>(ws + L.X);
  double* C = reinterpret_cast<double*>(ws + L.C);
  double* ug = reinterpret_cast<double*>(ws + L.ug);
  int* gd = guard ? reinterpret_cast<int*>(ws + L.guard) : nullptr;
  so.workspace = ws + L.solve_ws;
  so.workspace_bytes = sw;
  const long long vsz = (long long)g.n * g.n * g.n;
  const double sigma = g.sigma;
  // Step 4a: right-hand sides and particular solutions
  hipLaunchKernelGGL(k_pks_rhs, dim3(grid1(vsz)), dim3(kB), 0, s, rho_in, c_in, b->m_plus, g.n,
                     g.h, dt, chi, sigma, b2, gd);
  DPM_TRY_HIP(hipGetLastError());
  // Step 5: Tr_gamma_in G f (written by the solve's last pass where it fuses, else gathered from
  // the solutions), least squares, densities
  const bool fuse = restrict_fusable(g, so);
  if (fuse) {
    double* tr = reinterpret_cast<double*>(ws + L.tr);
    const TraceOut to{b->idx_in, b->in_zoff, tr, b->n_in};
    DPM_TRY(aux_solve_impl(g, 2, b2, X, so, s, nullptr, nullptr, false, 0, nullptr, &to));
    qr_solve(b, 2, tr, C, s);
  } else {
    DPM_TRY(aux_solve_impl(g, 2, b2, X, so, s, nullptr));
    qr_solve_traces(b, 2, X, vsz, C, s);
  }
  hipLaunchKernelGGL(k_density, dim3(grid1(b->n_gamma)), dim3(kB), 0, s, b->basis, C,
                     b->n_basis, b->n_basis, b->n_gamma, ug);
  // Steps 6-7: Green's formula as one AP solve per species
  // b2 holds sigma 1_{M+} f, zero on M-: add the M- part (sigma - Lap_h)[u_gamma] in place
  minus_rhs(b, ug, 0, 2, b2, s);
  DPM_TRY_HIP(hipGetLastError());
  // restriction to N+ (and the stepper's finiteness guard): fused into the solve's last pass
  // where it is a plain FP64 plane-sweep solve, else its own kernel
  if (fuse) {
    const RestrictOut ro{b->n_plus, rho_out, c_out, gd};
    DPM_TRY(aux_solve_impl(g, 2, b2, X, so, s, info, nullptr, false, 0, &ro));
  } else {
    DPM_TRY(aux_solve_impl(g, 2, b2, X, so, s, info));
    hipLaunchKernelGGL(k_restrict, dim3(grid1(vsz)), dim3(kB), 0, s, X, b->n_plus, vsz, rho_out,
                       c_out, gd);
  }
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace

dpm_status step_impl(const dpm_bep* b, double dt, double chi, const double* rho_in,
                     const double* c_in, double* rho_out, double* c_out, const dpm_opts& o,
                     hipStream_t s, dpm_info* info) {
  return step_enqueue(b, dt, chi, rho_in, c_in, rho_out, c_out, o, s, info, false);
}

dpm_status stepper_create_impl(const dpm_bep* b, double dt, double chi, double* rho, double* c,
                               const dpm_opts& o, hipStream_t s, dpm_stepper** out) {
  size_t need = 0;
  DPM_TRY(step_workspace_impl(b, o, &need));
  if (o.workspace == nullptr || o.workspace_bytes < need) {
    set_error("dpm_stepper_create: workspace too small: %zu bytes given, %zu needed",
              o.workspace_bytes, need);
    return DPM_EINVAL;
  }
  size_t sw = 0;
  dpm_opts so = o;
  so.rhs_chunk = 2;  // both species in one launch: the size never depends on tuning
  DPM_TRY(workspace_size_impl(b->grid, 2, so, &sw));
  int* gd = reinterpret_cast<int*>(static_cast<char*>(o.workspace) + step_layout(b, sw).guard);
  if (timing_enabled()) {
    set_error("dpm_stepper_create: sweep timing is enabled; end it before capturing a step");
    return DPM_EINVAL;
  }
  const Plan* pl = nullptr;
  DPM_TRY(get_plan(b->grid.n, &pl));  // tables exist before capture: no allocation inside it

  hipStream_t cs = nullptr;
  DPM_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    set_error("dpm_stepper_create: hipStreamBeginCapture: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  const dpm_status st = step_enqueue(b, dt, chi, rho, c, rho, c, o, cs, nullptr, true);
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (st != DPM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error("dpm_stepper_create: graph capture: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  hipLaunchKernelGGL(k_guard_init, dim3(1), dim3(64), 0, s, gd);
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    set_error("dpm_stepper_create: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  auto* p = new dpm_stepper;
  p->bep = b;
  p->graph = graph;
  p->exec = exec;
  p->guard = gd;
  *out = p;
  return DPM_OK;
}

dpm_status stepper_run_impl(dpm_stepper* p, int nsteps, hipStream_t s) {
  for (int k = 0; k < nsteps; ++k) DPM_TRY_HIP(hipGraphLaunch(p->exec, s));
  p->steps_run += nsteps;
  return DPM_OK;
}

dpm_status stepper_first_nonfinite_impl(const dpm_stepper* p, hipStream_t s, int32_t* step) {
  int v = 0;
  DPM_TRY_HIP(hipMemcpyAsync(&v, p->guard + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  DPM_TRY_HIP(hipStreamSynchronize(s));
  *step = v == INT_MAX ? 0 : v;
  return DPM_OK;
}

void stepper_destroy_impl(dpm_stepper* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();  // replays still in flight finish before the graph goes
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

dpm_status cfl_scan_impl(const dpm_bep* b, const double* rho, const double* c, double* out2,
                         hipStream_t s) {
  const dpm_grid& g = b->grid;
  const long long vsz = (long long)g.n * g.n * g.n;
  auto* o = reinterpret_cast<unsigned long long*>(out2);
  hipLaunchKernelGGL(k_scan_init, dim3(1), dim3(64), 0, s, o);
  const unsigned nblk = grid1(vsz) < (unsigned)kScanBlocks ? grid1(vsz) : (unsigned)kScanBlocks;
  hipLaunchKernelGGL(k_cfl_scan, dim3(nblk), dim3(kB), 0, s, rho, c, b->m_plus, g.n, g.h, o);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

namespace {
// dpm_run's workspace: [step workspace | scan area (scanned maxima, rank pair) | rebuild scratch]
struct RunLayout {
  size_t scan, rebuild, total;
};
dpm_status run_layout(const dpm_bep* b, const dpm_opts& o, RunLayout* L) {
  size_t need = 0;
  DPM_TRY(step_workspace_impl(b, o, &need));
  L->scan = align_up(need, 256);
  L->rebuild = L->scan + 256;
  L->total = L->rebuild + align_up(rebuild_scratch_bytes(b), 256);
  return DPM_OK;
}
}  // namespace

dpm_status run_workspace_impl(const dpm_bep* b, const dpm_opts& o, size_t* bytes) {
  RunLayout L{};
  DPM_TRY(run_layout(b, o, &L));
  *bytes = L.total;
  return DPM_OK;
}

dpm_status run_impl(dpm_bep* b, const dpm_run_params& p, double* rho, double* c,
                    const dpm_opts& o, hipStream_t s, dpm_run_info* info, double* dt_hist,
                    uint8_t* rebuilt_hist) {
  RunLayout L{};
  DPM_TRY(run_layout(b, o, &L));
  if (o.workspace == nullptr || o.workspace_bytes < L.total) {
    set_error("dpm_run: workspace too small: %zu bytes given, %zu needed", o.workspace_bytes,
              L.total);
    return DPM_EINVAL;
  }
  char* wsb = static_cast<char*>(o.workspace);
  // scan[0..1]: scanned maxima; scan[2..3]: (min, max) |R_ii| of the last rebuild, read back
  // with the next scan, so a rebuild adds no synchronisation of its own
  double* scan = reinterpret_cast<double*>(wsb + L.scan);
  void* rscratch = wsb + L.rebuild;
  const size_t rbytes = L.total - L.rebuild;
  dpm_run_info r{};
  r.stop = DPM_RUN_MAXSTEPS;
  double t = 0.0, dt_prev = 1.0 / b->grid.sigma;
  double rho_prev = 0.0;  // max |rho| of the previous scan (none before the first)
  bool rank_pending = false;
  for (;;) {
    // Steps 3 and 8: the CFL-type bound and the size of rho, from the current state
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const bool more = t < p.t_final && r.steps < p.max_steps;
    if (more) DPM_TRY(cfl_scan_impl(b, rho, c, scan, s));
    if (more || rank_pending) {
      DPM_TRY_HIP(hipMemcpyAsync(v, scan, sizeof(v), hipMemcpyDeviceToHost, s));
      DPM_TRY_HIP(hipStreamSynchronize(s));
    }
    if (rank_pending) {
      rank_pending = false;
      b->rdiag_min = v[2];
      b->rdiag_max = v[3];
      DPM_TRY(rank_check(v[2], v[3]));
    }
    if (t >= p.t_final) { r.stop = DPM_RUN_TFINAL; break; }
    if (r.steps >= p.max_steps) { r.stop = DPM_RUN_MAXSTEPS; break; }
    r.grad_max = v[0];
    r.rho_max = v[1];
    if (!(std::isfinite(v[0]) && std::isfinite(v[1]))) { r.stop = DPM_RUN_NONFINITE; break; }
    if (v[1] > p.rho_cap) { r.stop = DPM_RUN_RHOCAP; break; }
    if (p.rho_jump_cap > 0.0 && r.steps > 0 && v[1] - rho_prev >= p.rho_jump_cap) {
      r.stop = DPM_RUN_RHOJUMP;
      break;
    }
    rho_prev = v[1];
    double dt = dt_prev;
    if (v[0] > 0.0) {
      const double dt_cfl = b->grid.h / (6.0 * p.chi * v[0]);
      if (dt_cfl < dt) dt = dt_cfl;
    }
    // Step 4b: a smaller step needs the matrix (and its QR) at the new sigma
    const bool rebuild = dt < dt_prev;
    if (rebuild) {
      b->grid.sigma = 1.0 / dt;
      DPM_TRY(factor_bep_enqueue(b, s, nullptr, rscratch, rbytes, scan + 2));
      rank_pending = true;
      ++r.rebuilds;
    }
    // Steps 4a-7 in place
    DPM_TRY(step_enqueue(b, dt, p.chi, rho, c, rho, c, o, s, nullptr, false));
    if (dt_hist) dt_hist[r.steps] = dt;
    if (rebuilt_hist) rebuilt_hist[r.steps] = rebuild ? 1 : 0;
    ++r.steps;
    t += dt;
    dt_prev = dt;
  }
  DPM_TRY_HIP(hipStreamSynchronize(s));
  r.t = t;
  r.dt = dt_prev;
  if (info) *info = r;
  return DPM_OK;
}

dpm_status gauss_state_impl(const dpm_bep* b, const dpm_geometry& geo, double amp, double rate,
                            const double* c3, double* out, hipStream_t s) {
  const dpm_grid& g = b->grid;
  const long long vsz = (long long)g.n * g.n * g.n;
  hipLaunchKernelGGL(k_gauss_nodes, dim3(grid1(vsz)), dim3(kB), 0, s, b->m_plus, g.n, g.h, g.x0,
                     amp, rate, c3[0], c3[1], c3[2], out);
  hipLaunchKernelGGL(k_gauss_gamma, dim3(grid1(b->n_gamma)), dim3(kB), 0, s, b->idx, b->n_gamma,
                     g.n, g.h, g.x0, to_dev(geo), amp, rate, c3[0], c3[1], c3[2], out);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace dpm
