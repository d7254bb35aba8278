// Per-axis DST-I sweeps of the auxiliary-problem solve on gfx950.
//
// The AP (sigma I - Lap_h) u = b with zero Dirichlet data is diagonalised by the orthonormal
// DST-I S (S = S^T = S^-1) along each axis: u = S3 D^-1 S3 b, D = sigma + lambda_kx + lambda_ky
// + lambda_kz.  One solve is five passes over the volume: forward x, forward y, the z pass,
// inverse y, inverse x.  The z pass (z_tri.hip) solves the tridiagonal system along z of each
// spectral column (kx, ky) instead of transforming z, scaling and transforming back; the
// sweeps here are the x and y transforms.
//
// Sweep layout.  A block moves a tile of W whole lines (W * sizeof(real) = 128 bytes of every
// row of the tile, so each global access is a run of 128 contiguous bytes) into LDS with a
// padded pitch per line, transforms every line in place in its own LDS slot and
// writes the tile back.  Line transforms are wave-local: the G threads of a line sit in one
// wavefront and synchronise with wavefront barriers only; the two block barriers per tile
// separate the cooperative load, the transforms and the store.
//
// The line transform itself (a DST-I through a half-length complex FFT) is in dst_line.h.
// Sines and twiddles come from one FP64-computed table, held in LDS or read through L1/L2.
//
// The first x sweep of a refinement step computes the FP64 residual b - (sigma - Lap_h) u on the
// fly; the last x sweep can add its result into u (u += c) and reduce max|c|, max|u|.
#include "dst_line.h"

namespace dpm {

namespace {

// FP64 sweeps at N = 127 and 255 read their tables from global memory (L1/L2 resident) and are
// compiled for 4 waves per SIMD: with at most 38.7 KB of LDS per block, 4 blocks share a CU.
// FP32 sweeps and N >= 511 (two blocks per CU at most) keep the tables in LDS.
template <typename T, int LOGM>
struct ZOcc {
  static constexpr bool gtab = sizeof(T) == 8 && Cfg<T, LOGM>::G % 8 == 0 && LOGM <= 8;
  static constexpr int waves = gtab ? 4 : 1;
};

template <typename T, int LOGM, int AX, int IN, int OUT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ZOcc<T, LOGM>::waves)))
void k_dst_pass(PassArgs p, int tiles, int nblocks) {
  static_assert(AX == AX_X || AX == AX_Y, "the z direction is the tridiagonal pass");
  using K = Cfg<T, LOGM>;
  constexpr bool GTAB = ZOcc<T, LOGM>::gtab;
  constexpr int M = K::M, N = K::N, G = K::G, W = K::W, P = K::P;
  constexpr long long VOL = (long long)N * N * N;
  constexpr int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  constexpr int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  constexpr long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  constexpr long long S_LINE = (AX == AX_X) ? N : 1;
  constexpr long long S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : (long long)N * N);

  __shared__ __align__(16) T tile[W * P];
  __shared__ __align__(16) T tab[GTAB ? 2 : 3 * M];
  __shared__ unsigned long long red[2][kBlock / 64];

  const int logical = xcd_remap(blockIdx.x, nblocks);
  const int rhs = logical / tiles;
  const int t = logical - rhs * tiles;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;  // converged: uniform exit
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;

  const int row = t / TILES_PER_ROW;
  const int ti = t - row * TILES_PER_ROW;
  const int line0 = ti * W;
  const int nlines = min(W, LINES_PER_ROW - line0);
  const long long base = (long long)rhs * VOL + (long long)row * S_OUTER + (long long)line0 * S_LINE;
  const int tid = threadIdx.x;

  {
    const T* gtab = static_cast<const T*>(p.tw);
    if constexpr (!GTAB) {
      constexpr int TP = (3 * M + kBlock - 1) / kBlock;
      T tv[TP];
#pragma unroll
      for (int i = 0; i < TP; ++i) tv[i] = gtab[min(tid + i * kBlock, 3 * M - 1)];
#pragma unroll
      for (int i = 0; i < TP; ++i)
        if (tid + i * kBlock < 3 * M) tab[tid + i * kBlock] = tv[i];
    }
  }

  // ------------------------------------------------------------------ load the tile
  // Thread -> (line w of the tile, first element j0); its i-th element is j = j0 + JPI*i.  Along
  // x the JPI lanes of a line read consecutive elements; along y and z the W lanes of an
  // element index read W adjacent lines.  Either way a wavefront reads runs of >= 128 bytes.
  // Each thread forms one 32-bit byte offset; the step i moves a uniform base pointer, so the
  // loop carries no per-element address arithmetic.  Only steps that can reach j >= N clamp.
  constexpr int JPI = kBlock / W;                       // element stride between steps
  constexpr bool LINEMAJOR = AX == AX_X;
  constexpr bool STEPMAP = !LINEMAJOR || JPI * (int)sizeof(T) >= 128;
  constexpr int NSTEP = (N + JPI - 1) / JPI;            // steps per thread
  constexpr int IFULL = N / JPI;                        // steps with every j < N
  // Along y and z (FP64, 16 lines of 16 elements per step) the lanes of each wavefront are
  // permuted so that every 16-lane LDS pass covers 8 lines x 2 adjacent elements: with the line
  // pitch even, 16 lines of one element would be an even lane stride, which the LDS serves
  // slower than odd strides (measured 12% per instruction).  A wavefront still reads and
  // writes the same 128-byte runs.
  constexpr bool PERM = !LINEMAJOR && W == 16 && JPI == 16;
  const int lq = tid & 63, wq = tid >> 6;
  const int w = LINEMAJOR ? tid / JPI : (PERM ? ((lq & 7) | (((lq >> 4) & 1) << 3)) : tid % W);
  const int j0 = LINEMAJOR ? tid % JPI
                           : (PERM ? ((((lq >> 3) & 1) | ((lq >> 5) << 1)) + 4 * wq) : tid / W);
  const int wl = min(w, nlines - 1);                    // lines past the tile's end reload one
  const unsigned off0 = (unsigned)(wl * (int)S_LINE + j0 * (int)S_ELEM) * (unsigned)sizeof(T);
  // last step, clamped to j <= N - 1, relative to that step's base like every other step (an
  // absolute element offset overflows 32 bits along z at N = 1023)
  constexpr int JLAST = JPI * (NSTEP - 1);
  const unsigned offl = (unsigned)(wl * (int)S_LINE + min(j0, N - 1 - JLAST) * (int)S_ELEM) *
                        (unsigned)sizeof(T);
  T* const lds0 = tile + w * P + j0 + 1;                // slot of step 0; step i adds JPI*i
  const int jl = min(j0 + JPI * (NSTEP - 1), N);        // last step's slot (N: unused line[M])
  // per-thread line coordinates (x sweep, residual mode)
  const int lny = (line0 + wl) % N, lnz = (line0 + wl) / N;
  (void)lny; (void)lnz;

  // PER / CH of the flat mapping (FP32 x sweeps)
  constexpr int PER = (W * N + kBlock - 1) / kBlock;
  constexpr int CHMAX = IN == IN_RESID ? 8 : (sizeof(T) == 4 ? 16 : 8);
  constexpr int CH = PER < CHMAX ? PER : CHMAX;
  const T* __restrict__ in_t = static_cast<const T*>(p.in) + base;
  const double* __restrict__ in_d = static_cast<const double*>(p.in) + base;

  if constexpr (STEPMAP) {
    constexpr int SCHMAX = IN == IN_RESID ? 4 : 8;
    constexpr int SCH = NSTEP < SCHMAX ? NSTEP : SCHMAX;  // steps in flight per chunk
#pragma unroll
    for (int c0 = 0; c0 < NSTEP; c0 += SCH) {
      T v[SCH];
#pragma unroll
      for (int k = 0; k < SCH; ++k) {
        const int i = c0 + k;
        if (i >= NSTEP) break;
        const unsigned off = i < IFULL ? off0 : offl;
        const long long step = (long long)i * JPI * S_ELEM;
        if constexpr (IN == IN_RESID) {
          // FP64 residual b - (sigma - Lap_h) u at (x, y, z) = (j, lny, lnz)
          const double* __restrict__ ub = p.u + base + step;
          const double* __restrict__ bb = p.b + base + step;
          const int x = i < IFULL ? j0 + JPI * i : min(j0 + JPI * i, N - 1);
          const double uc = ld(ub, off);
          const double rb = LOGM == 8 ? ld_nt(bb, off) : ld(bb, off);  // b: read once
          // neighbours move the (uniform) pointer, never the unsigned offset below zero
          const double a0 = x > 0 ? ld(ub - 1, off) : 0.0;
          const double a1 = x < N - 1 ? ld(ub + 1, off) : 0.0;
          const double a2 = lny > 0 ? ld(ub - N, off) : 0.0;
          const double a3 = lny < N - 1 ? ld(ub + N, off) : 0.0;
          const double a4 = lnz > 0 ? ld(ub - (long long)N * N, off) : 0.0;
          const double a5 = lnz < N - 1 ? ld(ub + (long long)N * N, off) : 0.0;
          v[k] = (T)(rb - (sig + 6.0 * p.inv_h2) * uc +
                     p.inv_h2 * ((a0 + a1) + (a2 + a3) + (a4 + a5)));
        } else if constexpr (IN == IN_F64) {
          v[k] = (T)ld(in_d + step, off);
        } else if constexpr (IN == IN_F64_STREAM) {
          v[k] = (T)ld_nt(in_d + step, off);
        } else if constexpr (IN == IN_STREAM) {
          v[k] = ld_nt(in_t + step, off);
        } else {
          v[k] = ld(in_t + step, off);
        }
      }
#pragma unroll
      for (int k = 0; k < SCH; ++k) {
        const int i = c0 + k;
        if (i >= NSTEP) break;
        if (i < IFULL) lds0[JPI * i] = v[k];
        else tile[w * P + jl + 1] = v[k];
      }
    }
  } else if constexpr (IN == IN_RESID) {
    // FP64 residual into narrow reals along x: each wavefront takes a run of consecutive lines
    // of the tile, one line at a time, lane l holding x = l + 64 s.  The line's base is
    // uniform, so every load is the saddr form at the lane's 32-bit offset (512-byte runs) and
    // the y and z neighbour tests are uniform.  Along the run the y neighbours slide: a line's
    // own values and its y - 1 neighbour are the previous line's y + 1 neighbour and own values
    // (reloaded at the run's start and where a new z plane begins).  The x neighbours come from
    // the adjacent lanes (across a step boundary from the previous or next step's end lane).
    constexpr int XS = (N + 63) / 64;                  // steps per line
    constexpr int NWV = kBlock / 64;                   // wavefronts per block
    constexpr int LPW = (W + NWV - 1) / NWV;           // lines per wavefront
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double a6 = sig + 6.0 * p.inv_h2;
    double uc[XS], un[XS];                             // this line, and its y + 1 neighbour
#pragma unroll 1
    for (int i = 0; i < LPW; ++i) {
      const int wl0 = wv * LPW + i;                    // uniform in the wavefront
      if (wl0 >= nlines) break;
      const int ln = line0 + wl0;
      const int z = ln / N;
      const int y = ln - z * N;
      const bool fresh = i == 0 || y == 0;             // no previous line of this plane held
      const double* __restrict__ ub = p.u + base + (long long)wl0 * N;
      const double* __restrict__ bb = p.b + base + (long long)wl0 * N;
      double rb[XS], ys[XS], zs[XS];
#pragma unroll
      for (int s2 = 0; s2 < XS; ++s2) {
        const int x = min(lane + 64 * s2, N - 1);       // the last step's spare lanes reload
        const unsigned off = (unsigned)x * 8u;
        double a2;
        if (fresh) {
          a2 = y > 0 ? ld(ub - N, off) : 0.0;           // pointer moves, never the offset
          uc[s2] = ld(ub, off);
        } else {
          a2 = uc[s2];
          uc[s2] = un[s2];
        }
        un[s2] = y < N - 1 ? ld(ub + N, off) : 0.0;
        rb[s2] = LOGM == 8 ? ld_nt(bb, off) : ld(bb, off);  // b: read once
        const double a4 = z > 0 ? ld(ub - (long long)N * N, off) : 0.0;
        const double a5 = z < N - 1 ? ld(ub + (long long)N * N, off) : 0.0;
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
        const double r = rb[s2] - a6 * uc[s2] + p.inv_h2 * ((a0 + a1) + ys[s2] + zs[s2]);
        if (x < N) tile[wl0 * P + x + 1] = (T)r;
      }
    }
  } else {
    // flat mapping: thread owns tile elements e = tid + i*kBlock (x lines, narrow reals)
    const int cnt = nlines * N;
#pragma unroll 1
    for (int c0 = 0; c0 < PER; c0 += CH) {
      T v[CH];
      {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = min(tid + (c0 + i) * kBlock, cnt - 1);
          if constexpr (IN == IN_F64) v[i] = (T)in_d[e];
          else if constexpr (IN == IN_F64_STREAM) v[i] = (T)__builtin_nontemporal_load(in_d + e);
          else if constexpr (IN == IN_STREAM) v[i] = __builtin_nontemporal_load(in_t + e);
          else v[i] = in_t[e];
        }
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int e = tid + (c0 + i) * kBlock;
        if (e < cnt) {
          const int ww = e / N;
          tile[ww * P + (e - ww * N) + 1] = v[i];
        }
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ transform the lines
  const int g = tid % G;
#pragma unroll 1
  for (int round = 0; round < K::ROUNDS; ++round) {
    const int l = round * K::LPR + tid / G;
    if (l < nlines) {  // uniform across the G threads of a line (all in one wavefront)
      T* line = tile + l * P;
      if constexpr (K::G % 8 == 0) {
        const T* gtab_k = static_cast<const T*>(p.tw);
        const T* ttab = GTAB ? gtab_k : tab;
        C2<T> o[K::V];
        C2<T>* ob = reinterpret_cast<C2<T>*>(line) + g;
        dst1_regs<T, LOGM, false>(line, g, ttab, gtab_k, o);
#pragma unroll
        for (int s2 = 0; s2 < K::V; ++s2) ob[s2 * G] = o[s2];
        wave_sync();
      } else {
        dst1_line<T, LOGM>(line, g, tab);
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ store the tile
  double cm = 0.0, um = 0.0;
  if constexpr (STEPMAP) {
    if (w < nlines) {
      T v[NSTEP];
#pragma unroll
      for (int i = 0; i < NSTEP; ++i) v[i] = i < IFULL ? lds0[JPI * i] : tile[w * P + jl + 1];
      double old[OUT == OUT_UPD ? NSTEP : 1];
      if constexpr (OUT == OUT_UPD) {
        // all reads of u before its first write (the stores may alias the reads)
#pragma unroll
        for (int i = 0; i < NSTEP; ++i)
          old[i] = ld(static_cast<const double*>(p.out) + base + (long long)i * JPI * S_ELEM,
                      i < IFULL ? off0 : offl);
      }
#pragma unroll
      for (int i = 0; i < NSTEP; ++i) {
        if (i >= IFULL && j0 + JPI * i >= N) break;
        const unsigned off = i < IFULL ? off0 : offl;
        const long long step = (long long)i * JPI * S_ELEM;
        if constexpr (OUT == OUT_UPD) {
          const double nu = old[i] + (double)v[i];
          st(static_cast<double*>(p.out) + base + step, off, nu);
          cm = fmax(cm, fabs((double)v[i]));
          um = fmax(um, fabs(nu));
        } else if constexpr (OUT == OUT_F64) {
          st(static_cast<double*>(p.out) + base + step, off, (double)v[i]);
          cm = fmax(cm, fabs((double)v[i]));
        } else {
          st(static_cast<T*>(p.out) + base + step, off, v[i]);
        }
      }
    }
  } else if constexpr (AX == AX_X) {
    const int cnt = nlines * N;
#pragma unroll 1
    for (int c0 = 0; c0 < PER; c0 += CH) {
      T v[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int e = min(tid + (c0 + i) * kBlock, cnt - 1);
        const int ww = e / N;
        v[i] = tile[ww * P + (e - ww * N) + 1];
      }
      if constexpr (OUT == OUT_UPD) {
        double* uo = static_cast<double*>(p.out) + base;
        double old[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) old[i] = uo[min(tid + (c0 + i) * kBlock, cnt - 1)];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = tid + (c0 + i) * kBlock;
          if (e < cnt) {
            const double nu = old[i] + (double)v[i];
            uo[e] = nu;
            cm = fmax(cm, fabs((double)v[i]));
            um = fmax(um, fabs(nu));
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = tid + (c0 + i) * kBlock;
          if (e < cnt) {
            if constexpr (OUT == OUT_F64) {
              (static_cast<double*>(p.out) + base)[e] = (double)v[i];
              cm = fmax(cm, fabs((double)v[i]));
            } else {
              (static_cast<T*>(p.out) + base)[e] = v[i];
            }
          }
        }
      }
    }
  }

  if constexpr (AX == AX_X && OUT != OUT_WS) {
    if (p.cmax != nullptr) {
      if constexpr (OUT != OUT_UPD) um = cm;  // the first solve's correction is u itself
      // block max of cm, um -> one atomicMax each (max is order independent: deterministic)
      for (int off = 32; off > 0; off >>= 1) {
        cm = fmax(cm, __shfl_xor(cm, off));
        um = fmax(um, __shfl_xor(um, off));
      }
      const int wid = tid >> 6;
      if ((tid & 63) == 0) {
        red[0][wid] = (unsigned long long)__double_as_longlong(cm);
        red[1][wid] = (unsigned long long)__double_as_longlong(um);
      }
      __syncthreads();
      if (tid == 0) {
        unsigned long long c = red[0][0], uu = red[1][0];
        for (int w2 = 1; w2 < kBlock / 64; ++w2) {
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
dpm_status launch_t(AxisKind ax, bool zpass, InKind in, OutKind out, const PassArgs& a,
                    int nrhs, hipStream_t s) {
  using K = Cfg<T, LOGM>;
  constexpr int N = K::N, W = K::W;
  const long long lines_per_row = (ax == AX_X) ? (long long)N * N : N;
  const long long rows = (ax == AX_X) ? 1 : N;
  const long long tiles = rows * ((lines_per_row + W - 1) / W);
  const long long nb = tiles * nrhs;
  if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
  dim3 grid((unsigned)nb), block(kBlock);
  const int ti = (int)tiles, nbi = (int)nb;
  if (zpass || ax == AX_Z) { set_error("the z direction is the tridiagonal pass"); return DPM_EINVAL; }
  if (ax == AX_X) {
    if (in == IN_WS && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_WS, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_F64 && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_F64, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if ((in == IN_STREAM || in == IN_F64_STREAM) && out == OUT_WS) {
      // streamed kinds exist at n = 255 (launch_dst_pass maps other sizes to the plain kinds)
      if constexpr (LOGM == 8) {
        if (in == IN_STREAM) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_STREAM, OUT_WS>), grid, block, 0, s, a, ti, nbi);
        else if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_F64_STREAM, OUT_WS>), grid, block, 0, s, a, ti, nbi);
        else { set_error("FP64 transforms read FP64 input as IN_STREAM"); return DPM_EINVAL; }
      } else {
        set_error("streamed input kind at n != 255");
        return DPM_EINVAL;
      }
    }
    else if (in == IN_RESID && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_RESID, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_WS && out == OUT_F64) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_WS, OUT_F64>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_WS && out == OUT_UPD) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, IN_WS, OUT_UPD>), grid, block, 0, s, a, ti, nbi);
    else { set_error("unsupported x sweep kind (%d,%d)", (int)in, (int)out); return DPM_EINVAL; }
  } else {
    if ((in != IN_WS && in != IN_STREAM) || out != OUT_WS) { set_error("unsupported y sweep kind"); return DPM_EINVAL; }
    if (in == IN_WS) {
      hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_Y, IN_WS, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    } else {
      // the split layout's first sweep
      if constexpr (LOGM == 8) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_Y, IN_STREAM, OUT_WS>), grid, block, 0, s, a, ti, nbi);
      else { set_error("streamed input kind at n != 255"); return DPM_EINVAL; }
    }
  }
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

template <typename T>
dpm_status launch_size(int n, AxisKind ax, bool zpass, InKind in, OutKind out, const PassArgs& a,
                       int nrhs, hipStream_t s) {
  switch (n) {
    case 7: return launch_t<T, 3>(ax, zpass, in, out, a, nrhs, s);
    case 15: return launch_t<T, 4>(ax, zpass, in, out, a, nrhs, s);
    case 31: return launch_t<T, 5>(ax, zpass, in, out, a, nrhs, s);
    case 63: return launch_t<T, 6>(ax, zpass, in, out, a, nrhs, s);
    case 127: return launch_t<T, 7>(ax, zpass, in, out, a, nrhs, s);
    case 255: return launch_t<T, 8>(ax, zpass, in, out, a, nrhs, s);
    case 511: return launch_t<T, 9>(ax, zpass, in, out, a, nrhs, s);
    case 1023: return launch_t<T, 10>(ax, zpass, in, out, a, nrhs, s);
    default: set_error("no FFT sweep for n = %d", n); return DPM_EINVAL;
  }
}

}  // namespace

dpm_status launch_dst_pass(int real_bytes, int n, AxisKind ax, bool zpass, InKind in,
                           OutKind out, const PassArgs& a, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  // streamed input at n = 255 only (the plain loads elsewhere)
  if (n != 255 && in == IN_STREAM) in = IN_WS;
  if (n != 255 && in == IN_F64_STREAM) in = IN_F64;
  if (real_bytes == 4) return launch_size<float>(n, ax, zpass, in, out, a, nrhs, s);
  // FP64 transforms: FP64 input is the native type
  if (in == IN_F64) in = IN_WS;
  if (in == IN_F64_STREAM) in = IN_STREAM;
  return launch_size<double>(n, ax, zpass, in, out, a, nrhs, s);
}

}  // namespace dpm
