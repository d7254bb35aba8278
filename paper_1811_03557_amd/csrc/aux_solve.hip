// Driver of the auxiliary-problem solve: sweep sequence, FP64 iterative refinement with a
// device-side stop test (no host synchronisation, fixed launch count), batching in chunks.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace dpm {

namespace {

// Per right-hand-side refinement state lives at the start of the workspace.
struct FlagLayout {
  size_t done, iters, cmax, umax, prev, est, sig, total;
};
FlagLayout flag_layout(int nrhs) {
  FlagLayout f;
  size_t o = 0;
  f.done = o; o = align_up(o + sizeof(int) * nrhs, 256);
  f.iters = o; o = align_up(o + sizeof(int) * nrhs, 256);
  f.cmax = o; o = align_up(o + 8 * nrhs, 256);
  f.umax = o; o = align_up(o + 8 * nrhs, 256);
  f.prev = o; o = align_up(o + 8 * nrhs, 256);
  f.est = o; o = align_up(o + 8 * nrhs, 256);
  f.sig = o; o = align_up(o + 8 * nrhs, 256);
  f.total = o;
  return f;
}

__global__ void k_flags_reset(SolveFlags f, int nrhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nrhs) {
    f.done[i] = 0;
    f.iters[i] = 0;
    f.cmax[i] = 0ull;
    f.umax[i] = 0ull;
    f.prev[i] = 0.0;
    f.est[i] = 1.0;
  }
}

// After solve k (k = 0: the first solve, whose "correction" is u itself): the error left after
// the update is estimated from the geometric contraction of the corrections,
// est_k = ||c_k||^2 / (||c_{k-1}|| ||u_k||); refinement stops once est_k <= 0.1 rtol.
__global__ void k_flags_check(SolveFlags f, int rhs0, int nb, int k, double rtol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int r = rhs0 + i;
  if (f.done[r]) return;
  const double c = __longlong_as_double((long long)f.cmax[r]);
  const double u = __longlong_as_double((long long)f.umax[r]);
  if (k > 0) {
    f.iters[r] = k;
    const double pc = f.prev[r];
    double est = (u > 0.0 && pc > 0.0) ? (c / u) * (c / pc) : (c == 0.0 ? 0.0 : 1.0);
    if (!(est == est)) est = 1.0;  // NaN: not converged
    f.est[r] = est;
    if (est <= 0.1 * rtol) f.done[r] = 1;
  } else {
    f.est[r] = 1.0;
  }
  f.prev[r] = c;
  f.cmax[r] = 0ull;
  f.umax[r] = 0ull;
}

// Right-hand sides per launch: the chunk's transform volumes total about the 256 MB Infinity
// Cache (rounded to the nearest count; measured at 255^3: 2 FP64 or 4 FP32 volumes per launch
// beat 1 and 3).
static int default_chunk(int n, int nrhs, int real_bytes) {
  const double vol = (double)n * n * n * real_bytes;
  int c = (int)std::lround(256.0e6 / vol);
  if (c < 1) c = 1;
  if (c > nrhs) c = nrhs;
  if (c > 65535) c = 65535;
  return c;
}

bool needs_ws(const dpm_opts& o) {
  if (o.prec == DPM_FP32) return o.io_fp64 != 0;
  if (o.prec == DPM_FP64) return o.max_refine > 0;
  if (o.prec == DPM_FP64_GEMM) return false;  // in place in u, like plain FP64
  return true;  // BF16X3: FP32 tile workspace
}

int real_bytes_of(const dpm_opts& o) {
  return (o.prec == DPM_FP64 || o.prec == DPM_FP64_GEMM) ? 8 : 4;
}

// Widths and sweep layouts recorded by the autotuner, per (device, n, precision, I/O type,
// refinement on/off).
using TuneKey = std::tuple<int, int, int, int, int>;
struct Tuned {
  int width;
  int sweeps;  // DPM_SWEEPS_AXIS, DPM_SWEEPS_PLANE or DPM_SWEEPS_SPLIT
  int zcols;   // columns per block of the z pass (0: the default)
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tuned;

TuneKey tune_key(int n, const dpm_opts& o) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return TuneKey(dev, n, o.prec, o.io_fp64 != 0, o.max_refine > 0);
}

Tuned tuned_entry(int n, const dpm_opts& o) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tuned.empty()) return Tuned{0, DPM_SWEEPS_AUTO, 0};  // nothing tuned: no device query
  const auto it = g_tuned.find(tune_key(n, o));
  return it == g_tuned.end() ? Tuned{0, DPM_SWEEPS_AUTO, 0} : it->second;
}
int tuned_width(int n, const dpm_opts& o) { return tuned_entry(n, o).width; }

}  // namespace

size_t flags_bytes(int nrhs) { return flag_layout(nrhs).total; }

// Right-hand sides per launch: opts->rhs_chunk if set, else the width the autotuner recorded for
// these options, else the default; never more than nrhs.
int rhs_chunk_of(const dpm_grid& g, int nrhs, const dpm_opts& o) {
  if (o.rhs_chunk > 0) return o.rhs_chunk < nrhs ? o.rhs_chunk : nrhs;
  const int t = tuned_width(g.n, o);
  if (t > 0) return t < nrhs ? t : nrhs;
  return default_chunk(g.n, nrhs, real_bytes_of(o));
}

dpm_status validate_grid(const dpm_grid* g) {
  if (!g) { set_error("grid is NULL"); return DPM_EINVAL; }
  if (g->n < 7 || g->n > 1023) { set_error("n = %d out of range [7, 1023]", g->n); return DPM_EINVAL; }
  if (!(g->h > 0.0) || !std::isfinite(g->h)) { set_error("h must be finite and > 0"); return DPM_EINVAL; }
  if (!(g->sigma >= 0.0) || !std::isfinite(g->sigma)) {
    set_error("sigma must be finite and >= 0");
    return DPM_EINVAL;
  }
  if (!std::isfinite(g->x0)) { set_error("x0 must be finite"); return DPM_EINVAL; }
  return DPM_OK;
}

dpm_status validate_opts(const dpm_grid& g, const dpm_opts* o) {
  if (!o) { set_error("opts is NULL"); return DPM_EINVAL; }
  if (o->prec != DPM_FP64 && o->prec != DPM_FP32 && o->prec != DPM_BF16X3 &&
      o->prec != DPM_FP64_GEMM) {
    set_error("unknown precision %d", o->prec);
    return DPM_EINVAL;
  }
  if (o->io_fp64 != 0 && o->io_fp64 != 1) { set_error("io_fp64 must be 0 or 1"); return DPM_EINVAL; }
  if (!o->io_fp64 && !(o->prec == DPM_FP32 && o->max_refine == 0)) {
    set_error("FP32 input/output requires prec = DPM_FP32 and max_refine = 0");
    return DPM_EINVAL;
  }
  if (o->max_refine < 0 || o->max_refine > 64) { set_error("max_refine out of range [0, 64]"); return DPM_EINVAL; }
  if (o->max_refine > 0 && !(o->rtol > 0.0 && std::isfinite(o->rtol))) {
    set_error("rtol must be finite and > 0 when refining");
    return DPM_EINVAL;
  }
  if (o->rhs_chunk < 0) { set_error("rhs_chunk must be >= 0"); return DPM_EINVAL; }
  if (o->sweeps != DPM_SWEEPS_AUTO && o->sweeps != DPM_SWEEPS_AXIS && o->sweeps != DPM_SWEEPS_PLANE &&
      o->sweeps != DPM_SWEEPS_SPLIT) {
    set_error("unknown sweep layout %d", o->sweeps);
    return DPM_EINVAL;
  }
  if (o->sweeps == DPM_SWEEPS_SPLIT &&
      (!((o->prec == DPM_FP64 && o->max_refine == 0) || (o->prec == DPM_FP32 && !o->io_fp64)) ||
       !split_size_supported(g.n))) {
    set_error("DPM_SWEEPS_SPLIT needs a plain solve (DPM_FP64 without refinement, or DPM_FP32 "
              "with FP32 I/O) and n in {255, 511} (n = %d)", g.n);
    return DPM_EINVAL;
  }
  if (o->sweeps == DPM_SWEEPS_PLANE &&
      (!(o->prec == DPM_FP64 || o->prec == DPM_FP32) || !xy_fusion_supported(g.n))) {
    set_error("DPM_SWEEPS_PLANE needs DPM_FP64 or DPM_FP32 transforms and n in {7, 15, 31, 63, "
              "127} (n = %d)", g.n);
    return DPM_EINVAL;
  }
  if (o->prec == DPM_FP64_GEMM) {
    if (!dense_size_supported(g.n) || o->max_refine != 0) {
      set_error("DPM_FP64_GEMM supports 7 <= n <= %d without refinement", kDenseMaxN);
      return DPM_EINVAL;
    }
  } else if (!fft_size_supported(g.n)) {
    // n + 1 not a power of two: the FP64 FFT form runs Bluestein's sweeps (plain solve)
    if (o->prec == DPM_FP64 && blue_size_supported(g.n)) {
      if (o->max_refine != 0) {
        set_error("n = %d (n + 1 not a power of two): DPM_FP64 runs without refinement", g.n);
        return DPM_EINVAL;
      }
    } else {
      set_error("n = %d: the FP32 and split-bf16 transforms need n + 1 a power of two; DPM_FP64 "
                "takes any 7 <= n <= %d (Bluestein), DPM_FP64_GEMM any 7 <= n <= %d", g.n,
                kBlueMaxN, kDenseMaxN);
      return DPM_EINVAL;
    }
  }
  if (o->prec == DPM_BF16X3 && g.n > 255) { set_error("DPM_BF16X3 supports n <= 255"); return DPM_EINVAL; }
  return DPM_OK;
}

// Transform forms of the sweeps: real FFT (dst_fft.hip), split-bf16 dense products on the
// bf16 matrix cores, FP64 dense products on the FP64 matrix cores.
enum { FORM_FFT = 0, FORM_BF16X3 = 1, FORM_F64MM = 2, FORM_BLUE = 3 };

int form_of(const dpm_grid& g, const dpm_opts& o) {
  if (o.prec == DPM_BF16X3) return FORM_BF16X3;
  if (o.prec == DPM_FP64_GEMM) return FORM_F64MM;
  return fft_size_supported(g.n) ? FORM_FFT : FORM_BLUE;
}

// The split layout serves the plain solves (no refinement): FP64, or FP32 with FP32 I/O.
static bool split_opts(const dpm_opts& o) {
  return (o.prec == DPM_FP64 && o.max_refine == 0) || (o.prec == DPM_FP32 && !o.io_fp64);
}

// Sweep layout of a solve (DPM_SWEEPS_AXIS, _PLANE or _SPLIT): the caller's, else the one the
// autotuner recorded for these options, else the plane sweeps where they exist (FFT form,
// n <= 127), the split layout at n = 511 (plain solves: measured 3% faster than the per-axis
// sweeps in FP64 and 16% in FP32 on MI355X, while at 255 the per-axis sweeps are 2-3% faster),
// the per-axis sweeps otherwise.  A layout that does not exist for the size falls back to the
// per-axis sweeps.
static int layout_of(const dpm_grid& g, const dpm_opts& o, int form) {
  if (form != FORM_FFT) return DPM_SWEEPS_AXIS;
  const bool plane_ok = xy_fusion_supported(g.n);
  const bool split_ok = split_size_supported(g.n) && split_opts(o);
  int want = o.sweeps;
  if (want == DPM_SWEEPS_AUTO) want = tuned_entry(g.n, o).sweeps;
  if (want == DPM_SWEEPS_AUTO)
    want = plane_ok ? DPM_SWEEPS_PLANE : (split_ok && g.n == 511) ? DPM_SWEEPS_SPLIT : DPM_SWEEPS_AXIS;
  if (want == DPM_SWEEPS_PLANE && plane_ok) return DPM_SWEEPS_PLANE;
  if (want == DPM_SWEEPS_SPLIT && split_ok) return DPM_SWEEPS_SPLIT;
  return DPM_SWEEPS_AXIS;
}

// Workspace bytes per right-hand side of a launch: the transform volume (when the solve needs
// one) and the split layout's separator planes.
static size_t ws_per_rhs(const dpm_grid& g, const dpm_opts& o, int layout) {
  const size_t vol = (size_t)g.n * g.n * g.n;
  size_t per = needs_ws(o) ? vol * (size_t)real_bytes_of(o) : 0;
  if (layout == DPM_SWEEPS_SPLIT) per += split_side_values(g.n) * (size_t)real_bytes_of(o);
  return per;
}

static size_t workspace_for_layout(const dpm_grid& g, int nrhs, const dpm_opts& o, int chunk,
                                   int layout) {
  const size_t vol = (size_t)g.n * g.n * g.n;
  size_t total = flags_bytes(nrhs);
  if (needs_ws(o)) total += align_up(vol * (size_t)chunk * (size_t)real_bytes_of(o), 256);
  if (layout == DPM_SWEEPS_SPLIT)
    total += align_up(split_side_values(g.n) * (size_t)chunk * (size_t)real_bytes_of(o), 256);
  return total;
}

size_t workspace_for_chunk(const dpm_grid& g, int nrhs, const dpm_opts& o, int chunk) {
  return workspace_for_layout(g, nrhs, o, chunk, layout_of(g, o, form_of(g, o)));
}

dpm_status workspace_size_impl(const dpm_grid& g, int nrhs, const dpm_opts& o, size_t* bytes) {
  *bytes = workspace_for_chunk(g, nrhs, o, rhs_chunk_of(g, nrhs, o));
  return DPM_OK;
}

// Width of the solve's sweep launches.  The width is read once per call (the autotuner may
// record a new one meanwhile) and, unless the caller fixed it (rhs_chunk > 0), narrowed to the
// widest one the caller's workspace holds: results do not depend on the width, and a workspace
// sized before a re-tune or a reset stays usable.  Returns 0 when not even one right-hand side
// per launch fits.
static int solve_chunk(const dpm_grid& g, int nrhs, const dpm_opts& o, int layout) {
  int chunk = rhs_chunk_of(g, nrhs, o);
  if (workspace_for_layout(g, nrhs, o, chunk, layout) <= o.workspace_bytes || o.rhs_chunk > 0)
    return chunk;
  const size_t fixed = flags_bytes(nrhs);
  if (o.workspace_bytes < fixed) return 0;
  const size_t per = ws_per_rhs(g, o, layout);
  if (per == 0) return chunk;
  const size_t fit = ((o.workspace_bytes - fixed) / 256 * 256) / per;
  return fit >= (size_t)chunk ? chunk : (int)fit;
}

// One solve of nb right-hand sides: five per-axis passes, two fused plane sweeps around the z
// pass (plane layout), or the y sweeps around the split z solve (split layout: x transforms
// fused with its elimination and reconstruction, zside its separator planes).  in_kind/out_kind
// select the first and last sweeps; src/dst are the first sweep's source and the last sweep's
// destination, ws the volume the middle sweeps work on.
static dpm_status solve_sweeps(const Plan* pl, int rb, const dpm_grid& g, InKind in_kind,
                              const void* src, OutKind out_kind, void* dst, void* ws,
                              const double* b, const double* u, const SolveFlags* fl, int rhs0,
                              int nb, bool gated, int form, const double* sig_rhs,
                              hipStream_t s, int layout, int zcols, void* zside,
                              const RestrictOut* ro = nullptr, const TraceOut* to = nullptr) {
  PassArgs a{};
  if (ro != nullptr) {
    a.mask = ro->mask;
    a.out1 = ro->out1;
    a.guard = ro->guard;
  }
  if (to != nullptr) {
    a.tr_idx = to->idx;
    a.tr_zoff = to->zoff;
    a.tr_out = to->out;
    a.tr_m = to->m;
  }
  a.sigma_rhs = sig_rhs;
  a.tw = rb == 4 ? (const void*)pl->tw_f : (const void*)pl->tw_d;
  a.lam_hat = pl->lam;
  a.sigma = g.sigma;
  a.inv_h2 = 1.0 / (g.h * g.h);
  a.done = gated ? fl->done : nullptr;
  a.rhs0 = rhs0;
  a.b = b;
  a.u = u;
  auto pass = [&](AxisKind ax, bool z, InKind ik, OutKind ok, const void* i, void* o, bool track,
                  bool first) {
    PassArgs q = a;
    q.in = i;
    q.out = o;
    q.cmax = track ? fl->cmax : nullptr;
    q.umax = track ? fl->umax : nullptr;
    const int kind = ax == AX_Y ? SW_Y : ax == AX_Z ? SW_Z
                   : ik == IN_RESID ? SW_X_RESID : ok == OUT_UPD ? SW_X_UPD
                   : first ? SW_X_FIRST : SW_X_LAST;
    const bool tm = timing_on(rhs0, nb);
    if (tm) timing_before(s);
    // FFT and Bluestein forms: the z pass is the tridiagonal solve in the (kx, ky) basis; the
    // four unnormalised in-plane transforms carry (sqrt(2/M)/2)^4 = 1/(4 M^2)
    const double m1 = g.n + 1.0;
    dpm_status st = z && (form == FORM_FFT || form == FORM_BLUE)
                      ? launch_z_tri(form == FORM_BLUE ? 8 : rb, g.n, q, 1.0 / (a.inv_h2 * 4.0 * m1 * m1), nb, s, zcols)
                  : form == FORM_BLUE ? launch_blue_pass(g.n, ax, z, q, pl, nb, s)
                  : form == FORM_BF16X3 ? launch_bf16x3_pass(g.n, ax, z, ik, ok, q, pl, nb, s)
                  : form == FORM_F64MM  ? launch_f64mm_pass(g.n, ax, z, q, pl, nb, s)
                                        : launch_dst_pass(rb, g.n, ax, z, ik, ok, q, nb, s);
    if (tm) timing_after(s, kind);
    return st;
  };
  // the caller's right-hand sides, read out of place by the first sweep, are streamed past the
  // caches (FFT form)
  const bool stream_first = form == FORM_FFT && src != ws;
  if (layout == DPM_SWEEPS_SPLIT) {
    // plain solves only: FP64 output is the transform type (FP32 output has FP32 transforms)
    if (in_kind == IN_F64 && rb == 8) in_kind = IN_WS;
    if (out_kind == OUT_F64 && rb == 8) out_kind = OUT_WS;
    if (in_kind != IN_WS || out_kind != OUT_WS || fl != nullptr) {
      set_error("split layout: plain solves only");
      return DPM_EINVAL;
    }
    const double m1 = g.n + 1.0;
    const double fscale = 1.0 / (a.inv_h2 * 4.0 * m1 * m1);
    auto split = [&](int phase, int kind) {
      PassArgs q = a;
      q.in = ws;
      q.out = ws;
      const bool tm = timing_on(rhs0, nb);
      if (tm) timing_before(s);
      dpm_status st = launch_split_pass(rb, g.n, phase, q, zside, fscale, nb, s);
      if (tm) timing_after(s, kind);
      return st;
    };
    DPM_TRY(pass(AX_Y, false, stream_first ? IN_STREAM : IN_WS, OUT_WS, src, ws, false, false));
    DPM_TRY(split(0, SW_XZ_FWD));
    DPM_TRY(split(1, SW_Z_SEP));
    DPM_TRY(split(2, SW_XZ_INV));
    DPM_TRY(pass(AX_Y, false, IN_WS, OUT_WS, ws, dst, false, false));
    return DPM_OK;
  }
  if (layout == DPM_SWEEPS_PLANE) {
    auto xy = [&](InKind ik, OutKind ok, const void* i, void* o, bool track, int kind) {
      PassArgs q = a;
      q.in = i;
      q.out = o;
      q.cmax = track ? fl->cmax : nullptr;
      q.umax = track ? fl->umax : nullptr;
      const bool tm = timing_on(rhs0, nb);
      if (tm) timing_before(s);
      dpm_status st = launch_xy_pass(rb, g.n, ik, ok, q, nb, s);
      if (tm) timing_after(s, kind);
      return st;
    };
    DPM_TRY(xy(in_kind, OUT_WS, src, ws, false, SW_XY_FWD));
    DPM_TRY(pass(AX_Z, true, IN_WS, OUT_WS, ws, ws, false, false));
    DPM_TRY(xy(IN_WS, out_kind, ws, dst, fl != nullptr, SW_XY_INV));
    return DPM_OK;
  }
  InKind first_in = in_kind;
  if (stream_first)
    first_in = in_kind == IN_WS ? IN_STREAM : in_kind == IN_F64 ? IN_F64_STREAM : in_kind;
  DPM_TRY(pass(AX_X, false, first_in, OUT_WS, src, ws, false, true));
  DPM_TRY(pass(AX_Y, false, IN_WS, OUT_WS, ws, ws, false, false));
  DPM_TRY(pass(AX_Z, true, IN_WS, OUT_WS, ws, ws, false, false));
  DPM_TRY(pass(AX_Y, false, IN_WS, OUT_WS, ws, ws, false, false));
  DPM_TRY(pass(AX_X, false, IN_WS, out_kind, ws, dst, fl != nullptr, false));
  return DPM_OK;
}

bool restrict_fusable(const dpm_grid& g, const dpm_opts& o) {
  const int form = form_of(g, o);
  return (o.prec == DPM_FP64 || (o.prec == DPM_FP32 && o.io_fp64)) && o.max_refine == 0 &&
         form == FORM_FFT && layout_of(g, o, form) == DPM_SWEEPS_PLANE && rhs_chunk_of(g, 2, o) >= 2;
}

dpm_status aux_solve_impl(const dpm_grid& g, int nrhs, const void* b, void* u, const dpm_opts& o,
                          hipStream_t s, dpm_info* info, const double* sigma_host, bool no_alloc,
                          int zcols, const RestrictOut* ro, const TraceOut* to) {
  // a fused restriction or trace output is the caller's decision (restrict_fusable, which reads
  // the recorded layout once): the solve then runs the plane sweeps without consulting the
  // autotuner's table again, so a re-tune in between cannot change the layout under it
  const bool fused_out = ro != nullptr || to != nullptr;
  if (fused_out && !(nrhs == 2 && (o.prec == DPM_FP64 || (o.prec == DPM_FP32 && o.io_fp64)) &&
                     o.max_refine == 0 && form_of(g, o) == FORM_FFT && xy_fusion_supported(g.n))) {
    set_error("fused restriction or traces: need an unrefined plane-sweep solve of two "
              "right-hand sides");
    return DPM_EINVAL;
  }
  if (ro != nullptr && to != nullptr) {
    set_error("fused restriction and traces in one solve");
    return DPM_EINVAL;
  }
  const Plan* pl = nullptr;
  DPM_TRY(no_alloc ? find_plan(g.n, &pl) : get_plan(g.n, &pl));
  const int rb = real_bytes_of(o);
  const int form = form_of(g, o);
  int layout = fused_out ? DPM_SWEEPS_PLANE : layout_of(g, o, form);
  if (zcols <= 0) zcols = tuned_entry(g.n, o).zcols;
  const bool ws_needed = needs_ws(o);
  int chunk = solve_chunk(g, nrhs, o, layout);
  if (layout == DPM_SWEEPS_SPLIT && o.sweeps == DPM_SWEEPS_AUTO &&
      (chunk <= 0 || workspace_for_layout(g, nrhs, o, chunk, layout) > o.workspace_bytes)) {
    // a workspace sized without the separator planes: the per-axis sweeps need none
    layout = DPM_SWEEPS_AXIS;
    chunk = solve_chunk(g, nrhs, o, layout);
  }
  const size_t need = workspace_for_layout(g, nrhs, o, chunk > 0 ? chunk : 1, layout);
  if (chunk <= 0 || o.workspace_bytes < need || (need > 0 && o.workspace == nullptr)) {
    set_error("workspace too small: %zu bytes given, %zu needed", o.workspace_bytes, need);
    return DPM_EINVAL;
  }
  char* wsb = static_cast<char*>(o.workspace);
  const FlagLayout fo = flag_layout(nrhs);
  SolveFlags fl;
  fl.done = reinterpret_cast<int*>(wsb + fo.done);
  fl.iters = reinterpret_cast<int*>(wsb + fo.iters);
  fl.cmax = reinterpret_cast<unsigned long long*>(wsb + fo.cmax);
  fl.umax = reinterpret_cast<unsigned long long*>(wsb + fo.umax);
  fl.prev = reinterpret_cast<double*>(wsb + fo.prev);
  fl.est = reinterpret_cast<double*>(wsb + fo.est);
  void* vol_ws = ws_needed ? (void*)(wsb + fo.total) : nullptr;
  void* zside = layout == DPM_SWEEPS_SPLIT
                    ? (void*)(wsb + fo.total +
                              (ws_needed ? align_up((size_t)g.n * g.n * g.n * (size_t)chunk * (size_t)rb, 256) : 0))
                    : nullptr;
  double* sig_dev = nullptr;
  if (sigma_host != nullptr) {
    sig_dev = reinterpret_cast<double*>(wsb + fo.sig);
    DPM_TRY_HIP(hipMemcpyAsync(sig_dev, sigma_host, sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
  }

  const size_t vol = (size_t)g.n * g.n * g.n;
  const size_t io_bytes = o.io_fp64 ? 8 : 4;
  const bool refine = o.max_refine > 0;
  // the flags (max-norms, stop test) serve refinement only: without it a solve tracks nothing
  const bool plain = !refine;
  if (!plain) {
    hipLaunchKernelGGL(k_flags_reset, dim3((nrhs + 255) / 256), dim3(256), 0, s, fl, nrhs);
    DPM_TRY_HIP(hipGetLastError());
  }

  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    const int nb = (nrhs - c0) < chunk ? (nrhs - c0) : chunk;
    const char* bc = static_cast<const char*>(b) + (size_t)c0 * vol * io_bytes;
    char* uc = static_cast<char*>(u) + (size_t)c0 * vol * io_bytes;
    if ((o.prec == DPM_FP64 && !refine) || o.prec == DPM_FP64_GEMM) {
      // FP64 transforms in place in u: no workspace traffic beyond u itself
      // (no max-norm tracking: only refinement uses it); with a fused restriction the last pass
      // writes the masked solutions to the caller's two volumes instead
      if ((ro != nullptr || to != nullptr) && chunk < 2) {
        set_error("fused restriction or traces: both right-hand sides must share one launch");
        return DPM_EINVAL;
      }
      DPM_TRY(solve_sweeps(pl, 8, g, IN_WS, bc, ro ? OUT_RESTRICT : to ? OUT_TRACE : OUT_F64, ro ? (void*)ro->out0 : uc,
                          uc, nullptr, nullptr, nullptr, c0, nb, false, form, sig_dev, s, layout,
                          zcols, zside, ro, to));
    } else if (o.prec == DPM_FP32 && !o.io_fp64) {
      DPM_TRY(solve_sweeps(pl, 4, g, IN_WS, bc, OUT_WS, uc, uc, nullptr, nullptr, nullptr, c0, nb,
                          false, form, sig_dev, s, layout, zcols, zside));
    } else {
      // reduced-precision (or FP64) transforms on the workspace, FP64 iterate in u
      const double* bd = reinterpret_cast<const double*>(bc);
      double* ud = reinterpret_cast<double*>(uc);
      if ((ro != nullptr || to != nullptr) && chunk < 2) {
        set_error("fused restriction or traces: both right-hand sides must share one launch");
        return DPM_EINVAL;
      }
      DPM_TRY(solve_sweeps(pl, rb, g, IN_F64, bc, ro ? OUT_RESTRICT : to ? OUT_TRACE : OUT_F64,
                          ro ? (void*)ro->out0 : uc, vol_ws, nullptr, nullptr,
                          refine ? &fl : nullptr, c0, nb, false, form, sig_dev, s, layout, zcols,
                          zside, ro, to));
      if (refine) {
        hipLaunchKernelGGL(k_flags_check, dim3((nb + 255) / 256), dim3(256), 0, s, fl, c0, nb, 0, o.rtol);
        DPM_TRY_HIP(hipGetLastError());
      }
      for (int k = 1; k <= o.max_refine; ++k) {
        DPM_TRY(solve_sweeps(pl, rb, g, IN_RESID, nullptr, OUT_UPD, uc, vol_ws, bd, ud, &fl, c0,
                            nb, true, form, sig_dev, s, layout, zcols, zside));
        hipLaunchKernelGGL(k_flags_check, dim3((nb + 255) / 256), dim3(256), 0, s, fl, c0, nb, k, o.rtol);
        DPM_TRY_HIP(hipGetLastError());
      }
    }
  }

  if (info && plain) {
    DPM_TRY_HIP(hipStreamSynchronize(s));
    info->refine_iters = 0;
    info->est_rel_err = 0.0;
  } else if (info) {
    DPM_TRY_HIP(hipStreamSynchronize(s));
    info->refine_iters = 0;
    info->est_rel_err = 0.0;
    bool all_done = true;
    // read back in fixed blocks of the per-RHS state (no host containers)
    constexpr int kB = 256;
    int it[kB], dn[kB];
    double est[kB];
    for (int r0 = 0; r0 < nrhs; r0 += kB) {
      const int m = nrhs - r0 < kB ? nrhs - r0 : kB;
      DPM_TRY_HIP(hipMemcpy(it, fl.iters + r0, sizeof(int) * m, hipMemcpyDeviceToHost));
      DPM_TRY_HIP(hipMemcpy(dn, fl.done + r0, sizeof(int) * m, hipMemcpyDeviceToHost));
      DPM_TRY_HIP(hipMemcpy(est, fl.est + r0, sizeof(double) * m, hipMemcpyDeviceToHost));
      for (int i = 0; i < m; ++i) {
        if (it[i] > info->refine_iters) info->refine_iters = it[i];
        if (est[i] > info->est_rel_err || !(est[i] == est[i])) info->est_rel_err = est[i];
        if (!dn[i]) all_done = false;
      }
    }
    if (!refine) info->est_rel_err = 0.0;
    if (refine && !all_done) {
      set_error("refinement did not reach rtol = %g in %d iterations (estimate %g)", o.rtol,
                o.max_refine, info->est_rel_err);
      return DPM_ENOTCONV;
    }
  }
  return DPM_OK;
}


// Autotuner of the launch shape.  The sweep kernels' tiles are fixed at compile time; chosen at
// run time are the number of right-hand sides a sweep launch carries and, where the fused plane
// sweeps exist, the sweep layout (five per-axis sweeps or three with the plane in LDS).  The
// width trades the launch count against how much of the batch's working set stays in the 256 MB
// Infinity Cache, the layout trades HBM passes against the plane sweep's occupancy (one 160 KB
// block per CU at n = 127 in FP64), so the best pair depends on the size, the precision and the
// chip, and is measured here.
const int kTuneWidths[kTuneMaxWidths] = {1, 2, 3, 4, 6, 8, 12, 16};

dpm_status autotune_impl(const dpm_grid& g, int nrhs, const dpm_opts& o, const void* b, void* u,
                         int reps, hipStream_t s, int32_t* widths, int32_t* sweeps,
                         int32_t* zcols, double* ms, int32_t* count, int32_t* best,
                         int32_t* best_sweeps, int32_t* best_zcols) {
  if (timing_enabled()) {
    set_error("dpm_autotune: sweep timing is enabled; end it before tuning");
    return DPM_EINVAL;
  }
  // with a transform workspace, stay at or below the default width, so that a workspace sized
  // for the default (before tuning) fits every width the tuner may record
  const int cap = needs_ws(o) ? default_chunk(g.n, 1 << 30, real_bytes_of(o)) : (1 << 30);
  // layouts to try: the caller's fixed one, else the per-axis sweeps and the fused layout of
  // the size (plane or split) where it exists
  const int form = form_of(g, o);
  int layouts[2] = {DPM_SWEEPS_AXIS, DPM_SWEEPS_PLANE};
  int nl = 1;
  if (o.sweeps != DPM_SWEEPS_AUTO) {
    layouts[0] = o.sweeps;
  } else if (form == FORM_FFT && xy_fusion_supported(g.n)) {
    nl = 2;
  } else if (form == FORM_FFT && split_size_supported(g.n) && split_opts(o)) {
    layouts[1] = DPM_SWEEPS_SPLIT;
    nl = 2;
  }
  // the recorded pair (if any) stays in force until the new one replaces it: the timed solves
  // below fix their width and layout explicitly, and concurrent solves keep the old one meanwhile
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    set_error("dpm_autotune: event creation failed");
    return DPM_EHIP;
  }
  // one candidate: an untimed solve (first touch, caches), then the best of `reps` timed ones
  auto time_solve = [&](const dpm_opts& ow, int zc, double* t) {
    dpm_status st = aux_solve_impl(g, nrhs, b, u, ow, s, nullptr, nullptr, false, zc);
    for (int r = 0; r < reps && st == DPM_OK; ++r) {
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess) st = aux_solve_impl(g, nrhs, b, u, ow, s, nullptr, nullptr, false, zc);
      if (st != DPM_OK) break;
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float el = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
      if (e != hipSuccess) {
        set_error("dpm_autotune: %s", hipGetErrorString(e));
        return DPM_EHIP;
      }
      if (r == 0 || el < *t) *t = el;
    }
    return st;
  };
  int n_out = 0, w_best = 0, l_best = DPM_SWEEPS_AXIS, z_best = 0;
  double t_best = 0.0;
  dpm_status st = DPM_OK;
  for (int li = 0; li < nl && st == DPM_OK; ++li) {
    for (int w : kTuneWidths) {
      if (w > nrhs || w > cap) continue;
      dpm_opts ow = o;
      ow.rhs_chunk = w;
      ow.sweeps = layouts[li];
      if (workspace_for_layout(g, nrhs, ow, w, layout_of(g, ow, form)) > o.workspace_bytes) continue;
      double t = 0.0;
      st = time_solve(ow, 0, &t);
      if (st != DPM_OK) break;
      if (widths) widths[n_out] = w;
      if (sweeps) sweeps[n_out] = layouts[li];
      if (zcols) zcols[n_out] = 0;
      if (ms) ms[n_out] = t;
      ++n_out;
      if (w_best == 0 || t < t_best) {  // ties keep the earlier candidate (narrower, per-axis)
        w_best = w;
        l_best = layouts[li];
        t_best = t;
      }
    }
  }
  // the z pass's columns per block (FFT and Bluestein forms), at the winning width and layout;
  // the default (0) stays unless a column count is strictly faster (the split layout has no
  // z pass)
  if (st == DPM_OK && w_best > 0 && (form == FORM_FFT || form == FORM_BLUE) &&
      l_best != DPM_SWEEPS_SPLIT) {
    dpm_opts ow = o;
    ow.rhs_chunk = w_best;
    ow.sweeps = l_best;
    for (int zc : {16, 32, 64}) {
      if (!z_tri_cols_valid(g.n, zc)) continue;
      double t = 0.0;
      st = time_solve(ow, zc, &t);
      if (st != DPM_OK) break;
      if (widths) widths[n_out] = w_best;
      if (sweeps) sweeps[n_out] = l_best;
      if (zcols) zcols[n_out] = zc;
      if (ms) ms[n_out] = t;
      ++n_out;
      if (t < t_best) {
        z_best = zc;
        t_best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DPM_OK) return st;
  if (w_best == 0) {
    set_error("dpm_autotune: the workspace (%zu bytes) fits no candidate width", o.workspace_bytes);
    return DPM_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key(g.n, o)] = Tuned{w_best, l_best, z_best};
  }
  if (count) *count = n_out;
  if (best) *best = w_best;
  if (best_sweeps) *best_sweeps = l_best;
  if (best_zcols) *best_zcols = z_best;
  return DPM_OK;
}

void autotune_reset() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

}  // namespace dpm
