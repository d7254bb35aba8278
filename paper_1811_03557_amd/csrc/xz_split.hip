// Split layout of the FFT-form solve at n = 255 and 511: four passes over the volume instead of
// five, by cutting the tridiagonal z solve (z_tri.hip) into its three parts and fusing the two
// large ones with the x transforms.
//
// The z solve of a spectral column (kx, ky) is segment-local except for the small system of its
// separators.  A block that holds 16 consecutive z-rows of one y, i.e. 16 whole x lines (each a
// run of n contiguous values), holds every segment-local quantity of the n columns (kx, ky) it
// transforms.  So, with the y transforms first:
//   1. forward y sweep (dst_fft.hip);
//   2. k_xz_fwd: a block owns rows z = 16 s ... 16 s + 15 of one y; it transforms the 16 lines
//      along x in LDS, then each thread takes a column kx of the tile and solves its segment's
//      15 rows, v = T_15^-1 f, writing v to the 15 rows and f_sep + v_last to the separator row;
//   3. k_z_sep: per column, the reduced system of the separators (it reads the separator rows
//      and the first row of every segment, 2 of every 16 rows, and writes the separator values
//      to a side array of (n + 1)/16 - 1 planes per right-hand side);
//   4. k_xz_inv: a block takes the tile of step 2 back, forms u = v + z_left p + z_right q and the
//      separator row u = z_right, transforms the lines along x and stores them;
//   5. inverse y sweep (dst_fft.hip).
// Steps 2 and 4 move one volume each way like any sweep; step 3 reads 2/16 and writes 1/16 of a
// volume, and step 4 reads 2/16 more from the side array: 66.5 bytes per point in FP64 against
// 80 for the five per-axis passes.
//
// Arithmetic per column: z_tri.hip's, term for term (segments of 16 rows with 15 unknowns and a
// separator, pivots in tau form from eps = h^2 sigma + lam_hat_kx + lam_hat_ky, the reduced
// M-matrix with its row excesses as sums of positive terms, p = q reversed).  Only the rounding
// of v and of the separator data to the transform precision between the passes is added (none
// in FP64).
#include "dst_line.h"

namespace dpm {

namespace {

constexpr int kSeg = 16;         // rows per segment: 15 unknowns and the separator
constexpr int kSepThreads = 256;  // threads per block of the separator pass

template <typename T, int LOGM>
struct SplitCfg {
  using K = Cfg<T, LOGM>;
  static constexpr int N = K::N, M = K::M, G = K::G, P = K::P;
  static constexpr int NSEG = M / kSeg;                         // segments per column
  static constexpr int NS = NSEG - 1;                           // separators per column
  // y rows per block (each z-row of the tile a run of YB n values): 1; two rows per block
  // (runs of 4 KB in FP64 at n = 255, 2 blocks of 512 threads per CU) measured no faster
  static constexpr int YB = 1;
  // block order: FP64 walks the segments of one y block consecutively, FP32 the y blocks of
  // one segment (each measured the faster order for its precision at n = 255)
  static constexpr bool SEG_INNER = sizeof(T) == 8;
  static constexpr int TB = kBlock * YB;                        // threads per block
  static constexpr int L = kSeg * YB;                           // lines per tile
  static constexpr int NYB = (N + YB - 1) / YB;                 // blocks per segment
  static constexpr int LPR = TB / G;                            // lines per transform round
  static constexpr int ROUNDS = (L + LPR - 1) / LPR;
  static constexpr int PER = (L * N + TB - 1) / TB;             // tile elements per thread
  static constexpr int CPT = (YB * N + TB - 1) / TB;            // columns per thread
  // FP64 at n = 255 reads its transform tables from global memory (L1/L2 resident) and runs
  // 4 waves per SIMD, like the per-axis sweeps; otherwise the tables sit in LDS
  static constexpr bool GTAB = sizeof(T) == 8 && G % 8 == 0 && LOGM <= 8;
  static constexpr int WAVES = GTAB ? 4 : 1;
};

// Pivots of T_15 = tridiag(-1, 2 + eps, -1) in tau form: c_k = 1/m_k with m_k = 1 + t_k,
// t_1 = 1 + eps, t_k = eps + t_{k-1}/m_{k-1}; returns 1 - a = t_15/m_15 (a = 1/m_15).
__device__ __forceinline__ double seg_pivots(double eps, double* cv) {
  double t = 1.0 + eps, at = 0.0;
#pragma unroll
  for (int k = 0; k < kSeg - 1; ++k) {
    const double ck = recip(1.0 + t);
    const double tc = t * ck;  // t_k / m_k = 1 - c_k
    cv[k] = ck;
    if (k == kSeg - 2) at = tc;
    t = eps + tc;
  }
  return at;
}

// q = T_15^-1 e_15: suffix products of the c_k, in place
__device__ __forceinline__ void seg_spike(double* cv) {
  double qn = 1.0;
#pragma unroll
  for (int k = kSeg - 2; k >= 0; --k) {
    qn *= cv[k];
    cv[k] = qn;
  }
}

// Tile of the fused passes: rows z = 16 s + r (r < nz) of the y rows y0 + yy (yy < ny) of one
// block, line l = 16 yy + r in LDS slot l (1-based: element x at slot x + 1), at
// row_off(l) = r n^2 + yy n from the block's base.  Lines outside (r >= nz or yy >= ny) load a
// copy of a valid one and are neither transformed nor stored.
// FP64: wavefront v moves lines v, v + WV, v + 2 WV, ... (WV wavefronts), each as 64 consecutive
// elements per instruction (512 contiguous bytes, the lane offset the only per-thread address;
// the last step clamps to x <= N - 1, its value parked in the unused slot M).  FP32: thread
// element e = tid + i TB is (line e / N, x = e % N), runs of 64 contiguous values.
struct TileShape {
  int nz, ny;  // valid rows of the segment, valid y rows of the block
};
__device__ __forceinline__ bool line_valid(int l, TileShape sh) {
  return (l & (kSeg - 1)) < sh.nz && (l >> 4) < sh.ny;
}

template <typename T, int LOGM>
__device__ __forceinline__ long long line_off(int l, TileShape sh) {
  constexpr long long N = SplitCfg<T, LOGM>::N;
  const int r = min(l & (kSeg - 1), sh.nz - 1);
  const int yy = min(l >> 4, sh.ny - 1);
  return (long long)r * N * N + (long long)yy * N;
}

template <typename T, int LOGM>
__device__ __forceinline__ void tile_load(const T* src, T* tile, TileShape sh) {
  using S = SplitCfg<T, LOGM>;
  constexpr int N = S::N, P = S::P, CH = 8, TB = S::TB;
  const int tid = threadIdx.x;
  if constexpr (sizeof(T) == 8) {
    constexpr int WV = TB / 64;                     // wavefronts per block
    constexpr int LPW = S::L / WV;                  // lines per wavefront
    constexpr int NSTEP = (N + 63) / 64, IFULL = N / 64;
    constexpr int NI = LPW * NSTEP;
    const int wv = tid >> 6, lane = tid & 63;
    const unsigned off0 = (unsigned)lane * 8u;
    const unsigned offl = (unsigned)min(lane, N - 1 - 64 * (NSTEP - 1)) * 8u;
#pragma unroll
    for (int c0 = 0; c0 < NI; c0 += CH) {
      T v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = c0 + k;
        if (i >= NI) break;
        const int l = wv + WV * (i / NSTEP), st = i % NSTEP;
        v[k] = ld(src + line_off<T, LOGM>(l, sh) + 64 * st, st < IFULL ? off0 : offl);
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = c0 + k;
        if (i >= NI) break;
        const int l = wv + WV * (i / NSTEP), st = i % NSTEP;
        tile[l * P + min(64 * st + lane, N) + 1] = v[k];
      }
    }
  } else {
#pragma unroll
    for (int c0 = 0; c0 < S::PER; c0 += CH) {
      T v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= S::PER) break;
        const int e = min(tid + (c0 + k) * TB, S::L * N - 1);
        const int l = e / N;
        const int x = e - l * N;
        v[k] = (src + line_off<T, LOGM>(l, sh))[x];
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (c0 + k >= S::PER) break;
        const int e = tid + (c0 + k) * TB;
        if (e < S::L * N) {
          const int l = e / N;
          tile[l * P + (e - l * N) + 1] = v[k];
        }
      }
    }
  }
}

template <typename T, int LOGM>
__device__ __forceinline__ void tile_store(T* dst, const T* tile, TileShape sh) {
  using S = SplitCfg<T, LOGM>;
  constexpr int N = S::N, P = S::P, TB = S::TB;
  const int tid = threadIdx.x;
  if constexpr (sizeof(T) == 8) {
    constexpr int WV = TB / 64, LPW = S::L / WV;
    constexpr int NSTEP = (N + 63) / 64, IFULL = N / 64;
    const int wv = tid >> 6, lane = tid & 63;
    const unsigned off0 = (unsigned)lane * 8u;
#pragma unroll
    for (int r = 0; r < LPW; ++r) {
      const int l = wv + WV * r;
      if (!line_valid(l, sh)) continue;  // uniform per wavefront
#pragma unroll
      for (int st = 0; st < NSTEP; ++st) {
        if (st >= IFULL && 64 * st + lane >= N) break;
        ::dpm::st(dst + line_off<T, LOGM>(l, sh) + 64 * st, off0, tile[l * P + 64 * st + lane + 1]);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
      const int e = tid + i * TB;
      if (e < S::L * N) {
        const int l = e / N;
        const int x = e - l * N;
        if (line_valid(l, sh)) (dst + line_off<T, LOGM>(l, sh))[x] = tile[l * P + x + 1];
      }
    }
  }
}

// DST-I along x of the tile's valid lines, in place (G threads per line, wave-local)
template <typename T, int LOGM>
__device__ __forceinline__ void tile_transform(T* tile, TileShape sh, const T* ttab, const T* gtab) {
  using S = SplitCfg<T, LOGM>;
  using K = typename S::K;
  constexpr int G = S::G, P = S::P;
  const int tid = threadIdx.x;
  const int g = tid % G;
#pragma unroll 1
  for (int round = 0; round < S::ROUNDS; ++round) {
    const int l = round * S::LPR + tid / G;
    if (l < S::L && line_valid(l, sh)) {  // uniform across the G threads of a line (one wavefront)
      T* line = tile + l * P;
      C2<T> o[K::V];
      C2<T>* ob = reinterpret_cast<C2<T>*>(line) + g;
      dst1_regs<T, LOGM, false>(line, g, ttab, gtab, o);
#pragma unroll
      for (int s = 0; s < K::V; ++s) ob[s * G] = o[s];
      wave_sync();
    }
  }
}

// Block -> (right-hand side, y block, segment), the segments of one y block consecutive
// (SEG_INNER) or the y blocks of one segment.
struct TileId {
  int rhs, seg, y0;
  TileShape sh;
};
template <typename T, int LOGM>
__device__ __forceinline__ TileId tile_id(int nblocks) {
  using S = SplitCfg<T, LOGM>;
  constexpr int PER_RHS = S::NYB * S::NSEG;
  const int logical = xcd_remap(blockIdx.x, nblocks);
  TileId t;
  t.rhs = logical / PER_RHS;
  const int r = logical - t.rhs * PER_RHS;
  int yb;
  if constexpr (S::SEG_INNER) {
    yb = r / S::NSEG;
    t.seg = r - yb * S::NSEG;
  } else {
    t.seg = r / S::NYB;
    yb = r - t.seg * S::NYB;
  }
  t.y0 = yb * S::YB;
  t.sh.nz = t.seg == S::NSEG - 1 ? kSeg - 1 : kSeg;
  t.sh.ny = min(S::YB, S::N - t.y0);
  return t;
}

template <typename T, int LOGM>
__global__ __launch_bounds__((SplitCfg<T, LOGM>::TB))
__attribute__((amdgpu_waves_per_eu(SplitCfg<T, LOGM>::WAVES)))
void k_xz_fwd(PassArgs p, int nblocks, double fscale) {
  using S = SplitCfg<T, LOGM>;
  constexpr int N = S::N, M = S::M, P = S::P, TB = S::TB;
  constexpr long long NN = (long long)N * N, VOL = NN * N;
  __shared__ __align__(16) T tile[S::L * P];
  __shared__ __align__(16) T tab[S::GTAB ? 2 : 3 * M];

  const TileId id = tile_id<T, LOGM>(nblocks);
  if (p.done != nullptr && p.done[p.rhs0 + id.rhs] != 0) return;  // converged: uniform exit
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + id.rhs] : p.sigma;
  const bool last = id.seg == S::NSEG - 1;
  const long long base = (long long)id.rhs * VOL + (long long)(id.seg * kSeg) * NN + (long long)id.y0 * N;
  const T* gtab = static_cast<const T*>(p.tw);
  const int tid = threadIdx.x;
  if constexpr (!S::GTAB)
    for (int i = tid; i < 3 * M; i += TB) tab[i] = gtab[i];
  tile_load<T, LOGM>(static_cast<const T*>(p.in) + base, tile, id.sh);
  __syncthreads();
  tile_transform<T, LOGM>(tile, id.sh, S::GTAB ? gtab : tab, gtab);
  __syncthreads();

  // segment-local solve of each column (kx, ky = y0 + yy): v = T_15^-1 f in place of f; the
  // separator row takes f_sep + v_last, the part of the separator's right-hand side this
  // segment holds
  const double h2 = 1.0 / p.inv_h2;
#pragma unroll 1
  for (int j = 0; j < S::CPT; ++j) {
    const int c = tid + j * TB;
    const int yy = c / N;
    if (yy >= id.sh.ny) break;
    const int kx = c - yy * N;
    const double eps = sig * h2 + (p.lam_hat[id.y0 + yy] + p.lam_hat[kx]);
    T* const col = tile + yy * kSeg * P + kx + 1;
    double cv[kSeg - 1];
    (void)seg_pivots(eps, cv);
    // forward elimination, then back substitution; in FP64 the forward values wait in the
    // column's LDS slots (exact), in FP32 in registers
    if constexpr (sizeof(T) == 8) {
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < kSeg - 1; ++k) {
        d = ((double)col[k * P] * fscale + d) * cv[k];
        col[k * P] = (T)d;
      }
      double vn = 0.0;
#pragma unroll
      for (int k = kSeg - 2; k >= 0; --k) {
        vn = (double)col[k * P] + cv[k] * vn;
        col[k * P] = (T)vn;
      }
      if (!last) col[(kSeg - 1) * P] = (T)((double)col[(kSeg - 1) * P] * fscale + (double)col[(kSeg - 2) * P]);
    } else {
      double f[kSeg - 1];
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < kSeg - 1; ++k) { d = ((double)col[k * P] * fscale + d) * cv[k]; f[k] = d; }
      double vn = 0.0;
#pragma unroll
      for (int k = kSeg - 2; k >= 0; --k) { vn = f[k] + cv[k] * vn; f[k] = vn; }
#pragma unroll
      for (int k = 0; k < kSeg - 1; ++k) col[k * P] = (T)f[k];
      if (!last) col[(kSeg - 1) * P] = (T)((double)col[(kSeg - 1) * P] * fscale + f[kSeg - 2]);
    }
  }
  __syncthreads();
  tile_store<T, LOGM>(static_cast<T*>(p.out) + base, tile, id.sh);
}

// Reduced system of the separators of column c = ky n + kx (one thread per column):
//   -b z_{j-1} + (2 + eps - a_j - a_{j+1}) z_j - b z_{j+1} = f_sep_j + v_last^j + v_first^{j+1},
// solved with pivots m_j = e_j + tau_j, tau_j = rho_j + b tau_{j-1}/m_{j-1}, row excesses
// rho = eps + (1 - a) at the ends and eps + (1 - a - b) = eps (1 + sum q) inside.
template <typename T, int LOGM>
__global__ __launch_bounds__(kSepThreads) void k_z_sep(PassArgs p, T* __restrict__ zs, int nblocks) {
  using S = SplitCfg<T, LOGM>;
  constexpr int N = S::N, NS = S::NS;
  constexpr long long NN = (long long)N * N, VOL = NN * N;
  constexpr int BPR = (int)((NN + kSepThreads - 1) / kSepThreads);  // blocks per right-hand side
  const int logical = xcd_remap(blockIdx.x, nblocks);
  const int rhs = logical / BPR;
  const int c = (logical - rhs * BPR) * kSepThreads + threadIdx.x;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;
  if (c >= NN) return;  // no barriers below
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;
  const T* __restrict__ v = static_cast<const T*>(p.in) + (long long)rhs * VOL + c;
  // right-hand sides: separator row 16 j + 15 (f_sep + v_last) plus the next segment's first row
  double r[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j)
    r[j] = (double)v[(long long)(kSeg * j + kSeg - 1) * NN] + (double)v[(long long)(kSeg * j + kSeg) * NN];
  const int ky = c / N;
  const int kx = c - ky * N;
  const double eps = sig * (1.0 / p.inv_h2) + (p.lam_hat[ky] + p.lam_hat[kx]);
  double cv[kSeg - 1];
  const double at = seg_pivots(eps, cv);
  seg_spike(cv);
  const double b = cv[0];
  double qs = 0.0;
#pragma unroll
  for (int k = 0; k < kSeg - 1; ++k) qs += cv[k];
  const double om = eps * qs;
  double im[NS];
  double tau = 0.0, g = 0.0, m1 = 0.0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const bool lsep = j + 1 == NS;
    const double rho = eps + (j == 0 ? at : om) + (lsep ? at : om);
    const double ej = lsep ? 0.0 : b;
    if (j == 0) { tau = rho; g = r[0]; }
    else { tau = rho + b * tau * m1; g = r[j] + b * m1 * g; }
    m1 = recip(ej + tau);
    r[j] = g;
    im[j] = m1;
  }
  T* __restrict__ zo = zs + (long long)rhs * NS * NN + c;
  double zn = 0.0;
#pragma unroll
  for (int j = NS - 1; j >= 0; --j) {
    const double ej = j + 1 == NS ? 0.0 : b;
    zn = (r[j] + ej * zn) * im[j];
    zo[(long long)j * NN] = (T)zn;
  }
}

template <typename T, int LOGM>
__global__ __launch_bounds__((SplitCfg<T, LOGM>::TB))
__attribute__((amdgpu_waves_per_eu(SplitCfg<T, LOGM>::WAVES)))
void k_xz_inv(PassArgs p, const T* __restrict__ zs, int nblocks) {
  using S = SplitCfg<T, LOGM>;
  constexpr int N = S::N, M = S::M, P = S::P, NS = S::NS, TB = S::TB;
  constexpr long long NN = (long long)N * N, VOL = NN * N;
  __shared__ __align__(16) T tile[S::L * P];
  __shared__ __align__(16) T tab[S::GTAB ? 2 : 3 * M];

  const TileId id = tile_id<T, LOGM>(nblocks);
  if (p.done != nullptr && p.done[p.rhs0 + id.rhs] != 0) return;
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + id.rhs] : p.sigma;
  const bool first = id.seg == 0;
  const bool last = id.seg == S::NSEG - 1;
  const long long base = (long long)id.rhs * VOL + (long long)(id.seg * kSeg) * NN + (long long)id.y0 * N;
  const T* gtab = static_cast<const T*>(p.tw);
  const int tid = threadIdx.x;
  if constexpr (!S::GTAB)
    for (int i = tid; i < 3 * M; i += TB) tab[i] = gtab[i];
  // the 15 rows of v (the separator row's content is no longer needed)
  tile_load<T, LOGM>(static_cast<const T*>(p.in) + base, tile, TileShape{kSeg - 1, id.sh.ny});
  __syncthreads();

  // u = v + z_left p + z_right q on the 15 rows, u = z_right on the separator row
  // (z_left = 0 for the first segment, z_right = 0 for the last)
  const T* zrow = zs + (long long)id.rhs * NS * NN + (long long)id.y0 * N;
  const double h2 = 1.0 / p.inv_h2;
#pragma unroll 1
  for (int j = 0; j < S::CPT; ++j) {
    const int c = tid + j * TB;
    const int yy = c / N;
    if (yy >= id.sh.ny) break;
    const int kx = c - yy * N;
    const double zl = first ? 0.0 : (double)zrow[(long long)(id.seg - 1) * NN + c];
    const double zr = last ? 0.0 : (double)zrow[(long long)id.seg * NN + c];
    const double eps = sig * h2 + (p.lam_hat[id.y0 + yy] + p.lam_hat[kx]);
    T* const col = tile + yy * kSeg * P + kx + 1;
    double cv[kSeg - 1];
    (void)seg_pivots(eps, cv);
    seg_spike(cv);
#pragma unroll
    for (int k = 0; k < kSeg - 1; ++k) {
      const double vk = (double)col[k * P];
      col[k * P] = (T)(vk + zl * cv[kSeg - 2 - k] + zr * cv[k]);
    }
    if (!last) col[(kSeg - 1) * P] = (T)zr;
  }
  __syncthreads();
  tile_transform<T, LOGM>(tile, id.sh, S::GTAB ? gtab : tab, gtab);
  __syncthreads();
  tile_store<T, LOGM>(static_cast<T*>(p.out) + base, tile, id.sh);
}

template <typename T, int LOGM>
dpm_status launch_split_t(int phase, const PassArgs& a, void* zside, double fscale, int nrhs,
                          hipStream_t s) {
  using S = SplitCfg<T, LOGM>;
  constexpr long long NN = (long long)S::N * S::N;
  if (phase == 1) {
    const long long bpr = (NN + kSepThreads - 1) / kSepThreads;
    const long long nb = bpr * nrhs;
    if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
    hipLaunchKernelGGL((k_z_sep<T, LOGM>), dim3((unsigned)nb), dim3(kSepThreads), 0, s, a,
                       static_cast<T*>(zside), (int)nb);
  } else {
    const long long nb = (long long)S::NYB * S::NSEG * nrhs;
    if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
    if (phase == 0)
      hipLaunchKernelGGL((k_xz_fwd<T, LOGM>), dim3((unsigned)nb), dim3(S::TB), 0, s, a, (int)nb, fscale);
    else
      hipLaunchKernelGGL((k_xz_inv<T, LOGM>), dim3((unsigned)nb), dim3(S::TB), 0, s, a,
                         static_cast<const T*>(zside), (int)nb);
  }
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace

bool split_size_supported(int n) { return n == 255 || n == 511; }

size_t split_side_values(int n) {
  const size_t nseg = (size_t)(n + 1) / kSeg;
  return (nseg - 1) * (size_t)n * (size_t)n;
}

dpm_status launch_split_pass(int real_bytes, int n, int phase, const PassArgs& a, void* zside,
                             double fscale, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (phase < 0 || phase > 2) { set_error("split pass phase %d", phase); return DPM_EINVAL; }
  if (zside == nullptr && phase != 0) { set_error("split pass: no side array"); return DPM_EINVAL; }
  if (real_bytes == 8) {
    if (n == 255) return launch_split_t<double, 8>(phase, a, zside, fscale, nrhs, s);
    if (n == 511) return launch_split_t<double, 9>(phase, a, zside, fscale, nrhs, s);
  } else if (real_bytes == 4) {
    if (n == 255) return launch_split_t<float, 8>(phase, a, zside, fscale, nrhs, s);
    if (n == 511) return launch_split_t<float, 9>(phase, a, zside, fscale, nrhs, s);
  }
  set_error("no split layout for n = %d", n);
  return DPM_EINVAL;
}

}  // namespace dpm
