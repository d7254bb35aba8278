// Internal declarations shared by the HIP sources of libdpm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <vector>

#include "dpm.h"

namespace dpm {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define DPM_TRY_HIP(call)                                                        \
  do {                                                                           \
    hipError_t e__ = (call);                                                     \
    if (e__ != hipSuccess) {                                                     \
      ::dpm::set_error("%s failed: %s", #call, hipGetErrorString(e__));          \
      return DPM_EHIP;                                                           \
    }                                                                            \
  } while (0)

#define DPM_TRY(expr)                \
  do {                               \
    dpm_status s__ = (expr);         \
    if (s__ != DPM_OK) return s__;   \
  } while (0)

// ---------------------------------------------------------------- small types
template <typename T>
struct C2 {
  T x, y;
};

// ---------------------------------------------------------------- per-(device, n) tables
struct Plan {
  int n = 0;
  int log2L = 0;             // complex FFT length L = 2(n+1) = 2^log2L
  // packed transform table (M = n + 1, H = M / 2), 3M reals:
  //   [ sin(pi j/M), j < M | e^{-2 pi i e/H}, e < H (complex) | e^{-2 pi i k/M}, k < H (complex) ]
  float* tw_f = nullptr;
  double* tw_d = nullptr;
  double* lam = nullptr;     // lambda_k = (4/h^2) sin^2(pi k / (2(n+1))) * h^2, k = 1..n
                             // (stored without the 1/h^2 factor: lam_hat = 4 sin^2(...))
  // split-bf16 dense sine matrix for the MFMA path: [Mpad][Mpad] bf16 hi and lo
  uint16_t* s_hi = nullptr;
  uint16_t* s_lo = nullptr;
  int mpad = 0;
  // the same matrix in FP64 for the FP64 matrix-core path (n <= kDenseMaxN, else null)
  double* s_d = nullptr;
  // Bluestein tables (n + 1 not a power of two, FP64 FFT form): FFT length L = 2^blue_logl >= 3n,
  // twiddles e^{-2 pi i e/L} (L complex), chirp w_j = e^{i pi j^2/(2(n+1))} (j <= n + 1,
  // complex), the chirp filter's transform FFT_L(c) / L (L complex); 0 / null otherwise
  int blue_logl = 0;
  double* blue_tw = nullptr;
  double* blue_w = nullptr;
  double* blue_ch = nullptr;
};

// Returns the plan of the current device for size n (creating it on first use).
dpm_status get_plan(int n, const Plan** out);
// The same, without creating it: DPM_EINVAL when dpm_prepare(n) (or a first solve of size n)
// has not run on the current device.  Allocates nothing.
dpm_status find_plan(int n, const Plan** out);

bool fft_size_supported(int n);  // n + 1 a power of two and 7 <= n <= 1023
// Bluestein sizes (FP64 FFT form for n + 1 not a power of two): 7 <= n <= kBlueMaxN (L = 2048
// at most, L >= 3n); blue_logl(n) = log2 L, or 0 when n is beyond the range.
constexpr int kBlueMaxN = 682;
int blue_logl(int n);
bool blue_size_supported(int n);
// Sizes of the dense (GEMM-form) FP64 sweeps: any 7 <= n <= kDenseMaxN (matrix padded to a
// multiple of 32, at most 544)
constexpr int kDenseMaxN = 543;
bool dense_size_supported(int n);

// ---------------------------------------------------------------- DST pass kernels
// IN_STREAM / IN_F64_STREAM: IN_WS / IN_F64 for a first sweep that reads the caller's
// right-hand sides out of place: they are read once, so non-temporal loads keep them from
// displacing the launch's working volumes from the 256 MB Infinity Cache.  Used at n = 255,
// where those volumes are about the cache's size (measured 3-5% faster solves); below, they fit
// beside the input, and at 511 one volume exceeds the cache four times over and the plain loads
// measure faster, so other sizes take the plain kinds.
enum InKind { IN_WS = 0, IN_F64 = 1, IN_RESID = 2, IN_STREAM = 3, IN_F64_STREAM = 4 };
// OUT_RESTRICT: FP64 output restricted to a mask, right-hand side 0 to `out`, 1 to `out1`
// (the DPM step's restriction to N+, fused into the last plane sweep of its second solve);
// OUT_TRACE: FP64 output and the values at listed nodes (the step's traces on gamma_in, from the
// last plane sweep of its first solve)
enum OutKind { OUT_WS = 0, OUT_F64 = 1, OUT_UPD = 2, OUT_RESTRICT = 3, OUT_TRACE = 4 };
enum AxisKind { AX_X = 0, AX_Y = 1, AX_Z = 2 };

struct PassArgs {
  const void* in;            // input volume (chunk base)
  void* out;                 // output volume (chunk base)
  const double* b;           // residual mode: right-hand sides (chunk base)
  const double* u;           // residual mode: current iterate (chunk base)
  const void* tw;            // twiddles of the transform precision
  const double* lam_hat;     // 4 sin^2(pi k/(2(n+1))), k = 1..n
  double sigma;
  const double* sigma_rhs;   // per right-hand side sigma (device, nullable: use sigma)
  double inv_h2;
  const int* done;           // per right-hand side: skip the whole pass when set (nullable)
  unsigned long long* cmax;  // per rhs: max |correction| (update/store passes, nullable)
  unsigned long long* umax;  // per rhs: max |u_new|
  int rhs0;                  // index of the chunk's first right-hand side in the batch
  const uint8_t* mask;       // OUT_RESTRICT: N^3 mask (1 keeps the value, 0 writes zero)
  double* out1;              // OUT_RESTRICT: output volume of right-hand side 1
  int* guard;                // OUT_RESTRICT: stepper guard (nullable): a non-finite output
                             // records guard[0] into guard[1] by atomic minimum
  // OUT_TRACE: the solution at listed nodes as well:
  // tr_out[r tr_m + i] = u_r[tr_idx[i]], the nodes of z-plane z being i in [tr_zoff[z], tr_zoff[z+1])
  const int32_t* tr_idx;
  const int32_t* tr_zoff;
  double* tr_out;
  int tr_m;
};

// Launch one sweep over `nrhs` consecutive volumes.  real_bytes = 4 (FP32) or 8 (FP64).
dpm_status launch_dst_pass(int real_bytes, int n, AxisKind ax, bool zpass, InKind in,
                           OutKind out, const PassArgs& a, int nrhs, hipStream_t s);

// Fused plane sweep (both in-plane transforms of each z-plane, plane in LDS) over `nrhs`
// consecutive volumes; n = 7, 15, 31, 63, 127.  The forward pass (input kinds) writes the
// spectral planes transposed, the inverse pass (output kinds) reads them so.
bool xy_fusion_supported(int n);
dpm_status launch_xy_pass(int real_bytes, int n, InKind in, OutKind out, const PassArgs& a,
                          int nrhs, hipStream_t s);

// Middle pass of the FFT-form solves: the tridiagonal solve along z of every spectral column
// (kx, ky), in place on the volume the forward x and y sweeps left (either plane order).
// fscale multiplies the input: h^2 times the normalisation of the four in-plane transforms.
// cols: columns per block (16, 32 or 64 with ceil((n + 1) / 16) * cols <= 1024), 0 = default.
bool z_tri_supported(int n);  // 1 <= n <= 1023
bool z_tri_cols_valid(int n, int cols);
dpm_status launch_z_tri(int real_bytes, int n, const PassArgs& a, double fscale, int nrhs,
                        hipStream_t s, int cols = 0);

// Split layout of the FFT-form solve (n = 255, 511; plain solves): the z solve cut into the
// segment-local elimination fused with the forward x transforms (phase 0), the separators'
// reduced system (phase 1, written to zside: split_side_values(n) reals per right-hand side)
// and the reconstruction fused with the inverse x transforms (phase 2), in place on the volume
// the forward y sweep left; fscale as for launch_z_tri.
bool split_size_supported(int n);
size_t split_side_values(int n);
dpm_status launch_split_pass(int real_bytes, int n, int phase, const PassArgs& a, void* zside,
                             double fscale, int nrhs, hipStream_t s);

// Bluestein DST-I sweep (FP64, n + 1 not a power of two; plain solve kinds only).
dpm_status launch_blue_pass(int n, AxisKind ax, bool zpass, const PassArgs& a, const Plan* pl,
                            int nrhs, hipStream_t s);

// ---------------------------------------------------------------- BF16x3 MFMA dense DST
dpm_status launch_bf16x3_pass(int n, AxisKind ax, bool zpass, InKind in, OutKind out,
                              const PassArgs& a, const Plan* plan, int nrhs, hipStream_t s);

// ---------------------------------------------------------------- FP64 matrix-core dense DST
dpm_status launch_f64mm_pass(int n, AxisKind ax, bool zpass, const PassArgs& a, const Plan* plan,
                             int nrhs, hipStream_t s);

// ---------------------------------------------------------------- measurement support
// Sweep kinds reported by dpm_timing_end.
enum SweepKind { SW_X_FIRST = 0, SW_Y = 1, SW_Z = 2, SW_X_LAST = 3, SW_X_RESID = 4, SW_X_UPD = 5,
                 SW_XY_FWD = 6, SW_XY_INV = 7, SW_XZ_FWD = 8, SW_Z_SEP = 9, SW_XZ_INV = 10,
                 SW_KINDS = 11 };
bool timing_enabled();
bool timing_on(int rhs0, int nb);
void timing_before(hipStream_t s);
void timing_after(hipStream_t s, int kind);

// ---------------------------------------------------------------- solver internals
struct SolveFlags {
  int* done;
  int* iters;
  unsigned long long* cmax;
  unsigned long long* umax;
  double* prev;  // ||c_{k-1}||_inf
  double* est;   // estimated relative error after the last update
};

size_t flags_bytes(int nrhs);
// no_alloc: take the plan with find_plan (never create it) and read `info` back without host
// containers; the caller passes the library's static scratch as the workspace.
// zcols > 0: the z pass's columns per block (the autotuner's candidates), else the recorded
// or default one.
// The DPM step's restriction to N+ fused into the solve's last pass (out0/out1 receive the two
// right-hand sides' solutions masked; u is not written).  Only where restrict_fusable holds: an
// FP64, or FP32-transform with FP64 I/O, solve without refinement of two right-hand sides in
// one plane-sweep launch.
struct RestrictOut {
  const uint8_t* mask;
  double* out0;
  double* out1;
  int* guard;
};
bool restrict_fusable(const dpm_grid& g, const dpm_opts& o);
// The solution's values at listed nodes (the DPM step's traces on gamma_in) written by the last
// pass of a solve as well, under the same conditions: out[r m + i] = u_r[idx[i]], idx ascending
// in linear index with zoff[z] the first entry in z-plane z.
struct TraceOut {
  const int32_t* idx;
  const int32_t* zoff;
  double* out;
  int m;
};
dpm_status aux_solve_impl(const dpm_grid& g, int nrhs, const void* b, void* u,
                          const dpm_opts& o, hipStream_t s, dpm_info* info,
                          const double* sigma_host = nullptr, bool no_alloc = false,
                          int zcols = 0, const RestrictOut* ro = nullptr,
                          const TraceOut* to = nullptr);
// Device scratch of aux_solve_batched_noalloc: kStaticScratchBytes per device, owned by the
// library for the life of the process (static_scratch.hip).  Returns its device address on the
// current device, looked up once per device.
constexpr size_t kStaticScratchBytes = DPM_NOALLOC_SCRATCH_BYTES;
dpm_status static_scratch(void** out);
// Right-hand sides per sweep launch that a solve of nrhs right-hand sides uses.
int rhs_chunk_of(const dpm_grid& g, int nrhs, const dpm_opts& o);
dpm_status workspace_size_impl(const dpm_grid& g, int nrhs, const dpm_opts& o, size_t* bytes);
// Workspace bytes of a solve of nrhs right-hand sides at `chunk` right-hand sides per launch.
size_t workspace_for_chunk(const dpm_grid& g, int nrhs, const dpm_opts& o, int chunk);
// Launch-shape autotuner (see dpm_autotune): candidate widths x sweep layouts, timing, the
// recorded pairs.
constexpr int kTuneMaxWidths = 8;
constexpr int kTuneZCols = 3;
constexpr int kTuneMaxCands = 2 * kTuneMaxWidths + kTuneZCols;
static_assert(kTuneMaxCands <= DPM_TUNE_MAX_CANDIDATES, "candidate arrays of the ABI");
dpm_status autotune_impl(const dpm_grid& g, int nrhs, const dpm_opts& o, const void* b, void* u,
                         int reps, hipStream_t s, int32_t* widths, int32_t* sweeps,
                         int32_t* zcols, double* ms, int32_t* count, int32_t* best,
                         int32_t* best_sweeps, int32_t* best_zcols);
void autotune_reset();
dpm_status validate_grid(const dpm_grid* g);
dpm_status validate_opts(const dpm_grid& g, const dpm_opts* o);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace dpm
