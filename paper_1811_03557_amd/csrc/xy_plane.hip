// Fused plane sweeps of the auxiliary-problem solve (n <= 127): both in-plane DST-Is of one
// z-plane in one pass over it.
//
// With the plane held in LDS, a solve reads and writes the volume three times instead of five:
//   forward plane sweep: b[z][y][x] -> DST_y DST_x b, stored transposed as B[z][kx][ky];
//   z pass (z_tri.hip) on B: the tridiagonal solve along z of every spectral column, which
//   equals forward DST along z, division by sigma + lambda_kx + lambda_ky + lambda_kz and
//   inverse DST along z;
//   inverse plane sweep: B[z][kx][ky] -> DST_x DST_y B = u[z][y][x].
// The z pass is symmetric in its two in-plane indices, so it runs unchanged on the transposed
// spectral planes.
//
// A block owns one plane: it loads the plane's N rows into LDS slots (one slot per row, the
// slot doubling as the row's padded FFT buffer), transforms every row in place, transposes the
// plane inside LDS, transforms the rows again (the former columns) and stores the plane.  Each
// wavefront owns 64/G rows (G threads per row) through load, transforms and store, so block
// barriers surround only the transpose.  At n = 127 the FP64 plane (127 slots of 158 doubles,
// 160.5 KB) fills the CU's LDS; the block has 1024 threads, 8 per row, and the first
// transform's results go from registers straight to their transposed slots.
//
// Input kinds: the volume in the transform precision, FP64 converted on load, or the FP64
// residual b - (sigma - Lap_h) u formed on load.  Output kinds: the volume in the transform
// precision, FP64, or the update u += c; the FP64 kinds reduce max|c| and max|u| per
// right-hand side for the refinement's stop test.
#include "dst_line.h"

namespace dpm {

namespace {

template <typename T, int LOGM>
struct XYCfg {
  using K = Cfg<T, LOGM>;
  static constexpr int N = K::N, M = K::M, G = K::G, P = K::P;
  static constexpr int RW = 64 / G;                       // rows per wavefront
  static constexpr int WAVES = (N + RW - 1) / RW;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int ROWS_MAX = RW < N ? RW : N;       // rows a wavefront holds at most
  static constexpr int KMAX = (ROWS_MAX * N + 63) / 64;   // elements per lane of those rows
  // rows of 127 (8 threads per row): the register-resident transform (FP64 also reads its
  // tables through L1/L2); otherwise tables in LDS and the in-slot transform
  static constexpr bool REGS = G % 8 == 0;
  static constexpr bool GTAB = REGS && sizeof(T) == 8;
  static constexpr size_t LDS = sizeof(T) * (size_t)N * P;
};

// Planes that fit the CU's LDS (160 KB) with at most 1024 threads.
template <typename T, int LOGM>
constexpr bool xy_supported() {
  return LOGM >= 3 && LOGM <= 7 && XYCfg<T, LOGM>::LDS <= 160 * 1024 &&
         XYCfg<T, LOGM>::THREADS <= 1024;
}

// Row ownership: wavefront w loads, transforms and stores rows [w RW, w RW + RW) of the plane
// (a contiguous run of the volume), so only the transpose needs block-wide barriers; the other
// phases of different wavefronts overlap (one wavefront loads while another transforms).
template <typename T, int LOGM, int IN, int OUT>
__global__ __launch_bounds__((XYCfg<T, LOGM>::THREADS))
void k_xy_pass(PassArgs p, int nblocks) {
  using X = XYCfg<T, LOGM>;
  using K = typename X::K;
  constexpr int N = X::N, M = X::M, G = X::G, P = X::P, TH = X::THREADS, RW = X::RW;
  constexpr int KMAX = X::KMAX;
  constexpr long long VOL = (long long)N * N * N;
  constexpr int NN = N * N;

  __shared__ __align__(16) T plane[N * P];
  __shared__ __align__(16) T tab[X::GTAB ? 2 : 3 * M];
  __shared__ unsigned long long red[2][TH / 64];

  const int logical = xcd_remap(blockIdx.x, nblocks);  // neighbouring planes share an XCD's L2
  const int rhs = logical / N;
  const int z = logical - rhs * N;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;  // converged: uniform exit
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;
  const long long base = (long long)rhs * VOL + (long long)z * NN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int row0 = (tid >> 6) * RW;                    // the wavefront's first row
  const int cnt = (N - row0 < RW ? N - row0 : RW) * N;  // its elements (rows x N)
  const long long wbase = base + (long long)row0 * N;  // contiguous in the volume
  T* const wplane = plane + row0 * P;
  const T* gtab = static_cast<const T*>(p.tw);

  if constexpr (!X::GTAB) {
    for (int i = tid; i < 3 * M; i += TH) tab[i] = gtab[i];
    __syncthreads();
  }

  // ------------------------------------------------------------------ load the rows
  if constexpr (IN == IN_RESID) {
    // FP64 residual b - (sigma - Lap_h) u of the wavefront's rows, one row at a time with lane l
    // holding x = l + 64 s: every load is the saddr form at a uniform row base, the x
    // neighbours come from the adjacent lanes (across a step boundary from the previous or next
    // step's end lane), and along the rows a row's own values and its y - 1 neighbour are the
    // previous row's loads.
    constexpr int XS = (N + 63) / 64;                  // steps per row
    const int r0 = __builtin_amdgcn_readfirstlane(row0);
    const int rows = __builtin_amdgcn_readfirstlane(cnt) / N;
    const double a6 = sig + 6.0 * p.inv_h2;
    double uc[XS], un[XS];                             // this row, and its y + 1 neighbour
#pragma unroll 1
    for (int r = 0; r < rows; ++r) {
      const int y = r0 + r;
      const double* __restrict__ ub = p.u + wbase + (long long)r * N;
      const double* __restrict__ bb = p.b + wbase + (long long)r * N;
      double rb[XS], ys[XS], zs[XS];
#pragma unroll
      for (int s2 = 0; s2 < XS; ++s2) {
        const int x = min(lane + 64 * s2, N - 1);       // the last step's spare lanes reload
        const unsigned off = (unsigned)x * 8u;
        double a2;
        if (r == 0) {
          a2 = y > 0 ? ld(ub - N, off) : 0.0;           // pointer moves, never the offset
          uc[s2] = ld(ub, off);
        } else {
          a2 = uc[s2];
          uc[s2] = un[s2];
        }
        un[s2] = y < N - 1 ? ld(ub + N, off) : 0.0;
        rb[s2] = ld(bb, off);
        const double a4 = z > 0 ? ld(ub - NN, off) : 0.0;
        const double a5 = z < N - 1 ? ld(ub + NN, off) : 0.0;
        ys[s2] = a2 + un[s2];
        zs[s2] = a4 + a5;
      }
#pragma unroll
      for (int s2 = 0; s2 < XS; ++s2) {
        const int x = lane + 64 * s2;
        const double lm = __shfl_up(uc[s2], 1);         // lane - 1 (lane 0 keeps its own)
        const double lp = __shfl_down(uc[s2], 1);       // lane + 1 (lane 63 keeps its own)
        const double prev = s2 > 0 ? lane_value(uc[s2 > 0 ? s2 - 1 : 0], 63) : 0.0;
        const double next = s2 < XS - 1 ? lane_value(uc[s2 < XS - 1 ? s2 + 1 : 0], 0) : 0.0;
        const double a0 = x == 0 ? 0.0 : (lane == 0 ? prev : lm);
        const double a1 = x >= N - 1 ? 0.0 : (lane == 63 ? next : lp);
        // the stencil's sum in the order (x pair) + (y pair) + (z pair)
        const double res = rb[s2] - a6 * uc[s2] + p.inv_h2 * ((a0 + a1) + ys[s2] + zs[s2]);
        if (x < N) wplane[r * P + x + 1] = (T)res;
      }
    }
  } else {
    constexpr int CH = 8;
#pragma unroll
    for (int c0 = 0; c0 < KMAX; c0 += CH) {
      T v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= KMAX) break;
        const int e = min(lane + (c0 + k) * 64, cnt - 1);
        {
          // wave-uniform base of the step (clamped into the wavefront's rows), one 32-bit lane
          // offset in [0, 63]
          const int sk = min(64 * (c0 + k), cnt - 1);
          if constexpr (IN == IN_F64)
            v[k] = (T)ld(static_cast<const double*>(p.in) + wbase + sk, (unsigned)(e - sk) * 8u);
          else
            v[k] = ld(static_cast<const T*>(p.in) + wbase + sk, (unsigned)(e - sk) * (unsigned)sizeof(T));
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= KMAX) break;
        const int e = lane + (c0 + k) * 64;
        if (e < cnt) {
          const int r = e / N;
          wplane[r * P + (e - r * N) + 1] = v[k];
        }
      }
    }
  }
  wave_sync();

  const int g = lane % G;
  const int l = row0 + lane / G;  // the row this lane transforms (all G lanes of a row agree)
  T* const line = plane + l * P;
  // ------------------------------------------------------------------ rows, transpose, rows
  if constexpr (X::REGS) {
    const T* ttab = X::GTAB ? gtab : tab;
    C2<T> o[K::V];
    if (l < N) dst1_regs<T, LOGM, false>(line, g, ttab, gtab, o);
    __syncthreads();  // every row's slot is free: write the results to their transposed places
    if (l < N) {
      // o[s] = (2 X_2k, 2 X_2k+1), k = g + s*G: element i of row l goes to row i - 1, slot l + 1
#pragma unroll
      for (int s = 0; s < K::V; ++s) {
        const int k = g + s * G;
        if (k > 0) plane[(2 * k - 1) * P + l + 1] = o[s].x;
        if (2 * k + 1 <= N) plane[(2 * k) * P + l + 1] = o[s].y;
      }
    }
    __syncthreads();
    if (l < N) {
      dst1_regs<T, LOGM, false>(line, g, ttab, gtab, o);
      C2<T>* ob = reinterpret_cast<C2<T>*>(line) + g;
#pragma unroll
      for (int s = 0; s < K::V; ++s) ob[s * G] = o[s];
    }
    wave_sync();
  } else {
    if (l < N) dst1_line<T, LOGM>(line, g, tab);
    __syncthreads();
    {
      // the wavefront's rows of the transposed plane: element (r, c) is (c, r) of the plane
      T v[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        const int e = min(lane + k * 64, cnt - 1);
        const int r = e / N;
        v[k] = plane[(e - r * N) * P + row0 + r + 1];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        const int e = lane + k * 64;
        if (e < cnt) {
          const int r = e / N;
          wplane[r * P + (e - r * N) + 1] = v[k];
        }
      }
    }
    wave_sync();
    if (l < N) dst1_line<T, LOGM>(line, g, tab);
    wave_sync();
  }

  // ------------------------------------------------------------------ store the rows
  double cm = 0.0, um = 0.0;
  bool bad = false;  // OUT_RESTRICT: a non-finite output in this thread
  // OUT_RESTRICT: the right-hand side's own output volume, addressed within the plane
  double* const rout = OUT == OUT_RESTRICT ? (rhs == 0 ? static_cast<double*>(p.out) : p.out1) : nullptr;
  const long long lbase = (long long)z * NN + (long long)row0 * N;  // wavefront's rows, no rhs offset
  {
    constexpr int CH = 8;
#pragma unroll
    for (int c0 = 0; c0 < KMAX; c0 += CH) {
      T v[CH];
      double old[OUT == OUT_UPD ? CH : 1];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= KMAX) break;
        const int e = min(lane + (c0 + k) * 64, cnt - 1);
        const int r = e / N;
        v[k] = wplane[r * P + (e - r * N) + 1];
        if constexpr (OUT == OUT_UPD) {
          const int sk = min(64 * (c0 + k), cnt - 1);
          old[k] = ld(static_cast<const double*>(p.out) + wbase + sk, (unsigned)(e - sk) * 8u);
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= KMAX) break;
        const int e = lane + (c0 + k) * 64;
        if (e >= cnt) break;
        const long long sb = wbase + 64 * (c0 + k);  // wave-uniform base of the step (e < cnt)
        if constexpr (OUT == OUT_UPD) {
          const double nu = old[k] + (double)v[k];
          st(static_cast<double*>(p.out) + sb, (unsigned)lane * 8u, nu);
          cm = fmax(cm, fabs((double)v[k]));
          um = fmax(um, fabs(nu));
        } else if constexpr (OUT == OUT_F64 || OUT == OUT_TRACE) {
          st(static_cast<double*>(p.out) + sb, (unsigned)lane * 8u, (double)v[k]);
          cm = fmax(cm, fabs((double)v[k]));
        } else if constexpr (OUT == OUT_RESTRICT) {
          const long long rb = lbase + 64 * (c0 + k);
          const double vr = p.mask[rb + lane] ? (double)v[k] : 0.0;
          st(rout + rb, (unsigned)lane * 8u, vr);
          bad |= !isfinite(vr);
        } else {
          st(static_cast<T*>(p.out) + sb, (unsigned)lane * (unsigned)sizeof(T), v[k]);
        }
      }
    }
  }

  if constexpr (OUT == OUT_TRACE) {
    {
      // the solution at the listed nodes of this plane: every wavefront's final rows sit in LDS
      // once all have passed the barrier
      __syncthreads();
      const int i1 = p.tr_zoff[z + 1];
      for (int i = p.tr_zoff[z] + tid; i < i1; i += TH) {
        const int ep = p.tr_idx[i] - z * NN;
        const int y = ep / N;
        p.tr_out[(long long)(p.rhs0 + rhs) * p.tr_m + i] = (double)plane[y * P + (ep - y * N) + 1];
      }
    }
  }
  if constexpr (OUT == OUT_RESTRICT) {
    // a non-finite output records the current step number (guard[0]) into guard[1]: one
    // atomic per block that holds one, skipped once the step is recorded
    if (p.guard != nullptr && __syncthreads_or(bad) && tid == 0) {
      const int step = p.guard[0];
      if (p.guard[1] > step) atomicMin(&p.guard[1], step);
    }
  } else if constexpr (OUT != OUT_WS && OUT != OUT_TRACE) {
    if (p.cmax != nullptr) {
      if constexpr (OUT != OUT_UPD) um = cm;  // the first solve's correction is u itself
      // block max of cm, um -> one atomicMax each (max is order independent: deterministic)
      for (int off = 32; off > 0; off >>= 1) {
        cm = fmax(cm, __shfl_xor(cm, off));
        um = fmax(um, __shfl_xor(um, off));
      }
      const int wid = tid >> 6;
      if (lane == 0) {
        red[0][wid] = (unsigned long long)__double_as_longlong(cm);
        red[1][wid] = (unsigned long long)__double_as_longlong(um);
      }
      __syncthreads();
      if (tid == 0) {
        unsigned long long c = red[0][0], uu = red[1][0];
        for (int w2 = 1; w2 < TH / 64; ++w2) {
          c = c > red[0][w2] ? c : red[0][w2];
          uu = uu > red[1][w2] ? uu : red[1][w2];
        }
        atomicMax(p.cmax + p.rhs0 + rhs, c);
        atomicMax(p.umax + p.rhs0 + rhs, uu);
      }
    }
  }
}

template <typename T, int LOGM>
dpm_status launch_xy_t(InKind in, OutKind out, const PassArgs& a, int nrhs, hipStream_t s) {
  if constexpr (!xy_supported<T, LOGM>()) {
    (void)in; (void)out; (void)a; (void)nrhs; (void)s;
    set_error("no fused plane sweep for this size and precision");
    return DPM_EINVAL;
  } else {
    using X = XYCfg<T, LOGM>;
    const long long nb = (long long)X::N * nrhs;
    if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
    dim3 grid((unsigned)nb), block(X::THREADS);
    const int nbi = (int)nb;
    if (in == IN_WS && out == OUT_WS) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_WS, OUT_WS>), grid, block, 0, s, a, nbi);
    else if (in == IN_F64 && out == OUT_WS) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_F64, OUT_WS>), grid, block, 0, s, a, nbi);
    else if (in == IN_RESID && out == OUT_WS) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_RESID, OUT_WS>), grid, block, 0, s, a, nbi);
    else if (in == IN_WS && out == OUT_F64) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_WS, OUT_F64>), grid, block, 0, s, a, nbi);
    else if (in == IN_WS && out == OUT_UPD) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_WS, OUT_UPD>), grid, block, 0, s, a, nbi);
    else if (in == IN_WS && out == OUT_RESTRICT) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_WS, OUT_RESTRICT>), grid, block, 0, s, a, nbi);
    else if (in == IN_WS && out == OUT_TRACE) hipLaunchKernelGGL((k_xy_pass<T, LOGM, IN_WS, OUT_TRACE>), grid, block, 0, s, a, nbi);
    else { set_error("unsupported plane sweep kind (%d,%d)", (int)in, (int)out); return DPM_EINVAL; }
    DPM_TRY_HIP(hipGetLastError());
    return DPM_OK;
  }
}

template <typename T>
dpm_status launch_xy_size(int n, InKind in, OutKind out, const PassArgs& a, int nrhs,
                          hipStream_t s) {
  switch (n) {
    case 7: return launch_xy_t<T, 3>(in, out, a, nrhs, s);
    case 15: return launch_xy_t<T, 4>(in, out, a, nrhs, s);
    case 31: return launch_xy_t<T, 5>(in, out, a, nrhs, s);
    case 63: return launch_xy_t<T, 6>(in, out, a, nrhs, s);
    case 127: return launch_xy_t<T, 7>(in, out, a, nrhs, s);
    default: set_error("no fused plane sweep for n = %d", n); return DPM_EINVAL;
  }
}

}  // namespace

bool xy_fusion_supported(int n) { return n == 7 || n == 15 || n == 31 || n == 63 || n == 127; }

dpm_status launch_xy_pass(int real_bytes, int n, InKind in, OutKind out, const PassArgs& a,
                          int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (real_bytes == 4) return launch_xy_size<float>(n, in, out, a, nrhs, s);
  if (in == IN_F64) in = IN_WS;  // FP64 transforms: FP64 input is the native type
  return launch_xy_size<double>(n, in, out, a, nrhs, s);
}

}  // namespace dpm
