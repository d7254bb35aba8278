// Per-axis DST-I sweeps as dense FP64 products on the matrix cores (the "GEMM form" of the
// auxiliary-problem solve, the comparison to the FFT form of dst_fft.hip).
//
// A line x (N values, any 7 <= N <= 543, zero-padded to K = MP, a multiple of 32) is transformed
// as X = S x with S the orthonormal DST-I matrix (symmetric, S S = I); unlike the FFT form, N + 1
// need not be a power of two.  A block owns a tile of W = 32 lines, kept
// in LDS as [line][k] FP64 with an odd pitch (MP + 1), so that 16 consecutive lines of one k fall
// in distinct banks.  D[k][w] = sum_j S[k][j] In[w][j] with v_mfma_f64_16x16x4f64: A = S (16 rows
// k by 4 columns j, read from the plan's matrix, L2 resident), B = In^T (4 rows j by 16 lines,
// from LDS).  Operand and result layout of the instruction for lane l and item v (checked on
// the device): A[l % 16][l / 16], B[l / 16][l % 16], D[4 v + l / 16][l % 16].  Each wave owns one
// 16-line column block and half of the 16-row blocks, so its B operand is read once per k step.
// The z sweep runs the forward product, the eigenvalue scaling and the inverse product.
#include "common.h"

namespace dpm {

namespace {

constexpr int kT = 256;   // threads per block (4 waves)
constexpr int kWL = 32;   // lines per tile

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int MPAD>
struct CfgD {
  static constexpr int MP = MPAD;                  // padded K: the plan's matrix pitch
  static constexpr int PB = MP + 1;                // LDS pitch of a line (odd)
  static constexpr int KB = MP / 16;               // 16-row blocks of the output
  static constexpr int WB = kWL / 16;              // 16-line blocks of the output
  static constexpr int WPB = 4 / WB;               // waves per line block
  static constexpr int TPW = KB / WPB;             // output tiles per wave
};

// acc[t] = (S In^T) on the tiles of this wave: line block wb = wave % WB, row blocks
// kb = wave / WB + WPB t.
template <int MPAD>
__device__ __forceinline__ void tile_gemm_d(const double* __restrict__ S, const double* in,
                                            f64x4* acc, int wave, int lane) {
  using C = CfgD<MPAD>;
  constexpr int MP = C::MP, PB = C::PB, TPW = C::TPW, WB = C::WB, WPB = C::WPB;
  const int r = lane & 15, q = lane >> 4;
  const int wb = wave % WB, kb0 = wave / WB;
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const double* sa = S + (kb0 * 16 + r) * MP + q;   // row kb0*16 + r, column q
  const double* ib = in + (wb * 16 + r) * PB + q;   // line wb*16 + r, element q
#pragma unroll 2
  for (int k0 = 0; k0 < MP; k0 += 4) {
    const double b = ib[k0];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const double a = sa[(WPB * t * 16) * MP + k0];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
}

// Writes the tiles of this wave to LDS as [line][k]; scaled by 1/(bxy_w + inv_h2 lam_hat[k])
// (zero for k >= N or lines past the tile) when SCALE.
template <int MPAD, bool SCALE>
__device__ __forceinline__ void tile_stage_d(const f64x4* acc, double* in, int wave, int lane,
                                             int N, int nlines, double bxy, double inv_h2,
                                             const double* __restrict__ lam_hat) {
  using C = CfgD<MPAD>;
  constexpr int PB = C::PB, TPW = C::TPW, WB = C::WB, WPB = C::WPB;
  const int r = lane & 15, q = lane >> 4;
  const int wb = wave % WB, kb0 = wave / WB;
  const int w = wb * 16 + r;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kb = kb0 + WPB * t;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = kb * 16 + 4 * v + q;
      double d = acc[t][v];
      if constexpr (SCALE)
        d = (k < N && w < nlines) ? d / (bxy + inv_h2 * lam_hat[k < N ? k : N - 1]) : 0.0;
      in[w * PB + k] = d;
    }
  }
}

template <int MPAD, int AX, bool ZPASS>
__global__ __launch_bounds__(kT) void k_f64mm_pass(PassArgs p, const double* __restrict__ S,
                                                   int N, int tiles) {
  using C = CfgD<MPAD>;
  constexpr int MP = C::MP, PB = C::PB, TPW = C::TPW;
  constexpr int W = kWL;
  const long long VOL = (long long)N * N * N;
  const int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  const int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  const long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  const long long S_LINE = (AX == AX_X) ? N : 1;
  const long long S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : (long long)N * N);
  __shared__ __align__(16) double in[W * PB];

  const int rhs = blockIdx.y;
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;
  const int t = blockIdx.x;
  if (t >= tiles) return;
  const int row = t / TILES_PER_ROW;
  const int ti = t - row * TILES_PER_ROW;
  const int line0 = ti * W;
  const int nlines = min(W, LINES_PER_ROW - line0);
  const long long base = (long long)rhs * VOL + (long long)row * S_OUTER + (long long)line0 * S_LINE;
  const double* __restrict__ src = static_cast<const double*>(p.in) + base;
  double* __restrict__ dst = static_cast<double*>(p.out) + base;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  // ---- load the tile: along x the lanes read consecutive elements of a line, along y and z
  //      32 adjacent lines of one element (256-byte runs); zero padding for k >= N and for
  //      lines past the tile.  CH elements per thread are in flight together.
  constexpr int TOT = W * MP;
  constexpr int CH = 8;
#pragma unroll 1
  for (int e0 = 0; e0 < TOT; e0 += CH * kT) {
    double v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = e0 + i * kT + tid;
      int w, j;
      if constexpr (AX == AX_X) { w = e / MP; j = e - w * MP; }
      else { j = e / W; w = e - j * W; }
      const bool ok = e < TOT && w < nlines && j < N;
      v[i] = ok ? src[(long long)w * S_LINE + (long long)j * S_ELEM] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = e0 + i * kT + tid;
      if (e < TOT) {
        int w, j;
        if constexpr (AX == AX_X) { w = e / MP; j = e - w * MP; }
        else { j = e / W; w = e - j * W; }
        in[w * PB + j] = v[i];
      }
    }
  }
  __syncthreads();

  f64x4 acc[TPW];
  tile_gemm_d<MPAD>(S, in, acc, wave, lane);
  __syncthreads();  // every wave has read the tile
  if constexpr (ZPASS) {
    const int w = (wave % C::WB) * 16 + (lane & 15);
    const double bxy = w < nlines ? sig + p.inv_h2 * (p.lam_hat[line0 + w] + p.lam_hat[row]) : 1.0;
    tile_stage_d<MPAD, true>(acc, in, wave, lane, N, nlines, bxy, p.inv_h2, p.lam_hat);
    __syncthreads();
    tile_gemm_d<MPAD>(S, in, acc, wave, lane);
    __syncthreads();
  }
  tile_stage_d<MPAD, false>(acc, in, wave, lane, N, nlines, 0.0, 0.0, nullptr);
  __syncthreads();

  // ---- store the tile with the load's mapping
  const int TOTO = W * N;
#pragma unroll 4
  for (int e = tid; e < TOTO; e += kT) {
    int w, j;
    if constexpr (AX == AX_X) { w = e / N; j = e - w * N; }
    else { j = e / W; w = e - j * W; }
    if (w < nlines) dst[(long long)w * S_LINE + (long long)j * S_ELEM] = in[w * PB + j];
  }
}

template <int MPAD>
dpm_status launch_d(int n, AxisKind ax, const PassArgs& a, const Plan* pl, int nrhs,
                    hipStream_t s) {
  if (pl->mpad != MPAD || pl->s_d == nullptr) {
    set_error("FP64 sine matrix missing or with pad %d, expected %d", pl->mpad, MPAD);
    return DPM_EINVAL;
  }
  const long long lines_per_row = (ax == AX_X) ? (long long)n * n : n;
  const long long rows = (ax == AX_X) ? 1 : n;
  const long long tiles = rows * ((lines_per_row + kWL - 1) / kWL);
  dim3 grid((unsigned)tiles, nrhs), block(kT);
  const int ti = (int)tiles;
  if (ax == AX_X)
    hipLaunchKernelGGL((k_f64mm_pass<MPAD, AX_X, false>), grid, block, 0, s, a, pl->s_d, n, ti);
  else if (ax == AX_Y)
    hipLaunchKernelGGL((k_f64mm_pass<MPAD, AX_Y, false>), grid, block, 0, s, a, pl->s_d, n, ti);
  else
    hipLaunchKernelGGL((k_f64mm_pass<MPAD, AX_Z, true>), grid, block, 0, s, a, pl->s_d, n, ti);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace

dpm_status launch_f64mm_pass(int n, AxisKind ax, bool zpass, const PassArgs& a, const Plan* pl,
                             int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (nrhs > 65535) { set_error("too many right-hand sides in one launch"); return DPM_EINVAL; }
  if ((ax == AX_Z) != zpass) { set_error("the fused scaling belongs to the z sweep"); return DPM_EINVAL; }
  if (a.cmax != nullptr || a.done != nullptr) {
    set_error("the FP64 GEMM sweeps serve the plain solve (no refinement)");
    return DPM_EINVAL;
  }
  if (!dense_size_supported(n)) {
    set_error("DPM_FP64_GEMM supports 7 <= n <= %d", kDenseMaxN);
    return DPM_EINVAL;
  }
  switch ((n + 31) / 32) {
    case 1: return launch_d<32>(n, ax, a, pl, nrhs, s);
    case 2: return launch_d<64>(n, ax, a, pl, nrhs, s);
    case 3: return launch_d<96>(n, ax, a, pl, nrhs, s);
    case 4: return launch_d<128>(n, ax, a, pl, nrhs, s);
    case 5: return launch_d<160>(n, ax, a, pl, nrhs, s);
    case 6: return launch_d<192>(n, ax, a, pl, nrhs, s);
    case 7: return launch_d<224>(n, ax, a, pl, nrhs, s);
    case 8: return launch_d<256>(n, ax, a, pl, nrhs, s);
    case 9: return launch_d<288>(n, ax, a, pl, nrhs, s);
    case 10: return launch_d<320>(n, ax, a, pl, nrhs, s);
    case 11: return launch_d<352>(n, ax, a, pl, nrhs, s);
    case 12: return launch_d<384>(n, ax, a, pl, nrhs, s);
    case 13: return launch_d<416>(n, ax, a, pl, nrhs, s);
    case 14: return launch_d<448>(n, ax, a, pl, nrhs, s);
    case 15: return launch_d<480>(n, ax, a, pl, nrhs, s);
    case 16: return launch_d<512>(n, ax, a, pl, nrhs, s);
    default: return launch_d<544>(n, ax, a, pl, nrhs, s);
  }
}

}  // namespace dpm
