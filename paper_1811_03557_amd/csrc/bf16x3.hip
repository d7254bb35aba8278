// Per-axis DST-I sweeps as dense GEMMs on the MFMA units, in split bf16 ("bf16x3").
//
// A line x (N <= 255 values, zero-padded to K = MP, a multiple of 32) is transformed as
// X = S x with S the orthonormal DST-I matrix (S = S^T).  Both S and x are split into bf16 pairs
// x = x_hi + x_lo (x_hi = RNE(x), x_lo = RNE(x - x_hi)) and the product is taken as
// S_hi x_hi + S_hi x_lo + S_lo x_hi with FP32 accumulation (the dropped S_lo x_lo term is
// ~2^-16 relative).  The z sweep runs forward GEMM, eigenvalue scaling, inverse GEMM.
//
// Layout: a block owns a tile of W = 64 lines; the split input sits in LDS as [line][k] bf16
// (hi and lo), the output is staged in LDS as [line][k] FP32 and stored like the FFT sweeps.
// GEMM: D[k][w] = sum_j S[k][j] In[w][j] with v_mfma_f32_16x16x32_bf16: A = S (rows k, read from
// the plan's bf16 matrices in L2), B = In^T (columns = lines, from LDS).  Lane l of a 16x16 output
// tile holds D[4 (l / 16) + v][l % 16], v = 0..3.
#include "common.h"

namespace dpm {

namespace {

constexpr int kB = 256;
constexpr int kW = 64;  // lines per tile

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;                       // round to nearest even
  lo = (__bf16)(x - (float)hi);
}

template <int LOGM>
struct CfgB {
  static constexpr int M = 1 << LOGM;
  static constexpr int N = M - 1;
  static constexpr int MP = M < 32 ? 32 : M;  // padded K (multiple of 32)
  static constexpr int PB = MP + 8;           // bf16 pitch of a line in LDS
  static constexpr int PF = MP + 4;           // FP32 pitch of a line in LDS (staging)
  static constexpr int KB = MP / 16;          // 16-row blocks of the output
  static constexpr int WB = kW / 16;          // 16-column blocks of the output
  static constexpr int TPW = (KB * WB + 3) / 4;  // output tiles per wave
};

// GEMM of the tile: acc[t] (tiles owned by this wave) = S * In^T from the split operands.
template <int LOGM>
__device__ __forceinline__ void tile_gemm(const __bf16* __restrict__ s_hi,
                                          const __bf16* __restrict__ s_lo, const __bf16* in_hi,
                                          const __bf16* in_lo, f32x4* acc, int wave, int lane) {
  using C = CfgB<LOGM>;
  constexpr int MP = C::MP, PB = C::PB, WB = C::WB, TPW = C::TPW;
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int r = lane & 15, g = lane >> 4;
#pragma unroll 1
  for (int k0 = 0; k0 < MP; k0 += 32) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= C::KB * WB) break;
      const int kb = tile / WB, wb = tile - kb * WB;
      const int off_s = (kb * 16 + r) * MP + k0 + 8 * g;
      const bf16x8 a_hi = *reinterpret_cast<const bf16x8*>(s_hi + off_s);
      const bf16x8 a_lo = *reinterpret_cast<const bf16x8*>(s_lo + off_s);
      const int off_b = (wb * 16 + r) * PB + k0 + 8 * g;
      const bf16x8 b_hi = *reinterpret_cast<const bf16x8*>(in_hi + off_b);
      const bf16x8 b_lo = *reinterpret_cast<const bf16x8*>(in_lo + off_b);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_hi, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_lo, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, b_hi, acc[t], 0, 0, 0);
    }
  }
}

template <int LOGM, int AX, bool ZPASS, int IN, int OUT>
__global__ __launch_bounds__(kB) void k_bf16x3_pass(PassArgs p, const __bf16* __restrict__ s_hi,
                                                    const __bf16* __restrict__ s_lo, int tiles) {
  using C = CfgB<LOGM>;
  constexpr int N = C::N, MP = C::MP, PB = C::PB, PF = C::PF, WB = C::WB, TPW = C::TPW;
  constexpr int W = kW;
  constexpr long long VOL = (long long)N * N * N;
  constexpr int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  constexpr int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  constexpr long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  constexpr long long S_LINE = (AX == AX_X) ? N : 1;
  constexpr int S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : N * N);
  // LDS: split input [W][PB] hi + lo, reused as FP32 staging [W][PF]
  constexpr int BYTES_IN = 2 * W * PB * 2;
  constexpr int BYTES_OUT = W * PF * 4;
  __shared__ __align__(16) unsigned char smem[BYTES_IN > BYTES_OUT ? BYTES_IN : BYTES_OUT];
  __bf16* in_hi = reinterpret_cast<__bf16*>(smem);
  __bf16* in_lo = in_hi + W * PB;
  float* stage = reinterpret_cast<float*>(smem);

  const int rhs = blockIdx.y;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;
  const int t = blockIdx.x;
  const int row = t / TILES_PER_ROW;
  const int ti = t - row * TILES_PER_ROW;
  const int line0 = ti * W;
  const int nlines = min(W, LINES_PER_ROW - line0);
  const long long base = (long long)rhs * VOL + (long long)row * S_OUTER + (long long)line0 * S_LINE;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  // ---- load the tile, split into bf16 hi/lo; zero padding (k >= N, lines >= nlines).
  //      CH elements per thread are loaded together before they are used.
  constexpr int TOT = W * MP;
  constexpr int CH = IN == IN_RESID ? 4 : 16;
  auto index_of = [&](int e, int& w, int& j) {
    if constexpr (AX == AX_X) { w = e / MP; j = e - w * MP; }
    else { j = e / W; w = e - j * W; }
  };
#pragma unroll 1
  for (int e0 = 0; e0 < TOT; e0 += CH * kB) {
    float v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      int w, j;
      const int e = e0 + i * kB + tid;
      index_of(e, w, j);
      const bool ok = e < TOT && w < nlines && j < N;
      const int wc = ok ? w : 0, jc = ok ? j : 0;
      const long long gi = base + (long long)wc * S_LINE + (long long)jc * S_ELEM;
      if constexpr (IN == IN_F64) {
        const double x = static_cast<const double*>(p.in)[gi];
        v[i] = ok ? (float)x : 0.f;
      } else if constexpr (IN == IN_RESID) {
        const double* u = p.u;
        const int ln = line0 + wc;  // x sweep: line = (z, y), element = x
        const int z = ln / N, y = ln - z * N, x = jc;
        const double a0 = x > 0 ? u[gi - 1] : 0.0;
        const double a1 = x < N - 1 ? u[gi + 1] : 0.0;
        const double a2 = y > 0 ? u[gi - N] : 0.0;
        const double a3 = y < N - 1 ? u[gi + N] : 0.0;
        const double a4 = z > 0 ? u[gi - (long long)N * N] : 0.0;
        const double a5 = z < N - 1 ? u[gi + (long long)N * N] : 0.0;
        const double r = p.b[gi] - (sig + 6.0 * p.inv_h2) * u[gi] +
                         p.inv_h2 * ((a0 + a1) + (a2 + a3) + (a4 + a5));
        v[i] = ok ? (float)r : 0.f;
      } else {
        const float x = static_cast<const float*>(p.in)[gi];
        v[i] = ok ? x : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      int w, j;
      const int e = e0 + i * kB + tid;
      if (e < TOT) {
        index_of(e, w, j);
        __bf16 hi, lo;
        split_bf16(v[i], hi, lo);
        in_hi[w * PB + j] = hi;
        in_lo[w * PB + j] = lo;
      }
    }
  }
  __syncthreads();

  f32x4 acc[TPW];
  tile_gemm<LOGM>(s_hi, s_lo, in_hi, in_lo, acc, wave, lane);
  __syncthreads();  // every wave has read the split input

  if constexpr (ZPASS) {
    // scale D[k][w] by 1/(sigma + lambda_x + lambda_y + lambda_z), split again, inverse GEMM
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int tile = wave + 4 * tt;
      if (tile >= C::KB * WB) break;
      const int kb = tile / WB, wb = tile - kb * WB;
      const int w = wb * 16 + r;
      const double bxy = (w < nlines) ? sig + p.inv_h2 * (p.lam_hat[line0 + w] + p.lam_hat[row]) : 1.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kb * 16 + 4 * g + v;
        float d = 0.f;
        if (k < N && w < nlines) d = acc[tt][v] * (float)(1.0 / (bxy + p.inv_h2 * p.lam_hat[k]));
        __bf16 hi, lo;
        split_bf16(d, hi, lo);
        in_hi[w * PB + k] = hi;
        in_lo[w * PB + k] = lo;
      }
    }
    __syncthreads();
    tile_gemm<LOGM>(s_hi, s_lo, in_hi, in_lo, acc, wave, lane);
    __syncthreads();
  }

  // ---- stage D[k][w] as [w][k] FP32, then store
  {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int tile = wave + 4 * tt;
      if (tile >= C::KB * WB) break;
      const int kb = tile / WB, wb = tile - kb * WB;
#pragma unroll
      for (int v = 0; v < 4; ++v) stage[(wb * 16 + r) * PF + kb * 16 + 4 * g + v] = acc[tt][v];
    }
  }
  __syncthreads();
  double cm = 0.0, um = 0.0;
  {
    constexpr int TOTO = W * N;
    constexpr int CHO = 8;
#pragma unroll 1
    for (int e0 = 0; e0 < TOTO; e0 += CHO * kB) {
      double old[CHO];
      long long gis[CHO];
      bool oks[CHO];
#pragma unroll
      for (int i = 0; i < CHO; ++i) {
        int w, j;
        const int e = e0 + i * kB + tid;
        if constexpr (AX == AX_X) { w = e / N; j = e - w * N; }
        else { j = e / W; w = e - j * W; }
        oks[i] = e < TOTO && w < nlines;
        gis[i] = base + (long long)(oks[i] ? w : 0) * S_LINE + (long long)(oks[i] ? j : 0) * S_ELEM;
        if constexpr (OUT == OUT_UPD) old[i] = static_cast<const double*>(p.out)[gis[i]];
        else old[i] = stage[(oks[i] ? w : 0) * PF + (oks[i] ? j : 0)];
        if constexpr (OUT == OUT_UPD) old[i] += (double)stage[(oks[i] ? w : 0) * PF + (oks[i] ? j : 0)];
      }
#pragma unroll
      for (int i = 0; i < CHO; ++i) {
        if (!oks[i]) continue;
        if constexpr (OUT == OUT_UPD) {
          const double nu = old[i];
          static_cast<double*>(p.out)[gis[i]] = nu;
          um = fmax(um, fabs(nu));
        } else if constexpr (OUT == OUT_F64) {
          static_cast<double*>(p.out)[gis[i]] = old[i];
          cm = fmax(cm, fabs(old[i]));
        } else {
          static_cast<float*>(p.out)[gis[i]] = (float)old[i];
        }
      }
    }
    if constexpr (OUT == OUT_UPD) {
      // max |c| over the staged correction
      for (int e = tid; e < W * N; e += kB) {
        int w, j;
        if constexpr (AX == AX_X) { w = e / N; j = e - w * N; }
        else { j = e / W; w = e - j * W; }
        if (w < nlines) cm = fmax(cm, fabs((double)stage[w * PF + j]));
      }
    }
  }
  if constexpr (OUT != OUT_WS) {
    if (p.cmax != nullptr) {
      if constexpr (OUT != OUT_UPD) um = cm;
      for (int off = 32; off > 0; off >>= 1) {
        cm = fmax(cm, __shfl_xor(cm, off));
        um = fmax(um, __shfl_xor(um, off));
      }
      if (lane == 0) {
        atomicMax(p.cmax + p.rhs0 + rhs, (unsigned long long)__double_as_longlong(cm));
        atomicMax(p.umax + p.rhs0 + rhs, (unsigned long long)__double_as_longlong(um));
      }
    }
  }
}

template <int LOGM>
dpm_status launch_b(AxisKind ax, bool zpass, InKind in, OutKind out, const PassArgs& a,
                    const Plan* pl, int nrhs, hipStream_t s) {
  using C = CfgB<LOGM>;
  constexpr int N = C::N;
  if (pl->mpad != C::MP) {
    set_error("bf16 sine matrix has pad %d, expected %d", pl->mpad, C::MP);
    return DPM_EINVAL;
  }
  const long long lines_per_row = (ax == AX_X) ? (long long)N * N : N;
  const long long rows = (ax == AX_X) ? 1 : N;
  const long long tiles = rows * ((lines_per_row + kW - 1) / kW);
  dim3 grid((unsigned)tiles, nrhs), block(kB);
  const __bf16* sh = reinterpret_cast<const __bf16*>(pl->s_hi);
  const __bf16* sl = reinterpret_cast<const __bf16*>(pl->s_lo);
  const int ti = (int)tiles;
#define DPM_LAUNCHB(AXV, Z, INV, OUTV) \
  hipLaunchKernelGGL((k_bf16x3_pass<LOGM, AXV, Z, INV, OUTV>), grid, block, 0, s, a, sh, sl, ti)
  if (ax == AX_X) {
    if (in == IN_F64 && out == OUT_WS) DPM_LAUNCHB(AX_X, false, IN_F64, OUT_WS);
    else if (in == IN_RESID && out == OUT_WS) DPM_LAUNCHB(AX_X, false, IN_RESID, OUT_WS);
    else if (in == IN_WS && out == OUT_F64) DPM_LAUNCHB(AX_X, false, IN_WS, OUT_F64);
    else if (in == IN_WS && out == OUT_UPD) DPM_LAUNCHB(AX_X, false, IN_WS, OUT_UPD);
    else if (in == IN_WS && out == OUT_WS) DPM_LAUNCHB(AX_X, false, IN_WS, OUT_WS);
    else { set_error("unsupported bf16x3 x sweep kind"); return DPM_EINVAL; }
  } else if (ax == AX_Y) {
    DPM_LAUNCHB(AX_Y, false, IN_WS, OUT_WS);
  } else {
    DPM_LAUNCHB(AX_Z, true, IN_WS, OUT_WS);
  }
#undef DPM_LAUNCHB
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace

dpm_status launch_bf16x3_pass(int n, AxisKind ax, bool zpass, InKind in, OutKind out,
                              const PassArgs& a, const Plan* pl, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (nrhs > 65535) { set_error("too many right-hand sides in one launch"); return DPM_EINVAL; }
  if ((ax == AX_Z) != zpass) { set_error("the fused scaling belongs to the z sweep"); return DPM_EINVAL; }
  switch (n) {
    case 7: return launch_b<3>(ax, zpass, in, out, a, pl, nrhs, s);
    case 15: return launch_b<4>(ax, zpass, in, out, a, pl, nrhs, s);
    case 31: return launch_b<5>(ax, zpass, in, out, a, pl, nrhs, s);
    case 63: return launch_b<6>(ax, zpass, in, out, a, pl, nrhs, s);
    case 127: return launch_b<7>(ax, zpass, in, out, a, pl, nrhs, s);
    case 255: return launch_b<8>(ax, zpass, in, out, a, pl, nrhs, s);
    default: set_error("DPM_BF16X3 supports n = 7, 15, 31, 63, 127, 255"); return DPM_EINVAL;
  }
}

}  // namespace dpm
