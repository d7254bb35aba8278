// Per-axis DST-I sweeps for any line length N (N + 1 not a power of two): Bluestein's chirp-z
// method on power-of-two complex FFTs, FP64.
//
// With M = N + 1 and jk = (j^2 + k^2 - (k - j)^2) / 2,
//   Y_k = sum_{j=1..N} x_j e^{i pi j k / M} = w_k sum_j (x_j w_j) conj(w_{k-j}),
//   w_n = e^{i pi n^2 / (2M)},
// a linear convolution, computed as a cyclic one of length L (a power of two) through the FFT:
// y = IFFT_L( FFT_L(x w) . FFT_L(c) ), c_d = conj(w_d) placed at d mod L.  The DST-I is
// X_k = Im Y_k (sin = Im e^{i.}).  Two real lines x1, x2 share one transform as x = x1 + i x2:
// since x1 is real, Y1_{2M-k} = conj(Y1_k), and with w_{2M-k} = w_k,
//   Y1_k = (Y_k + conj Y_{2M-k}) / 2,  Y2_k = (Y_k - conj Y_{2M-k}) / (2i),
// so the outputs k = 1..N and 2M - k are needed: d = k - j spans [1 - N, 2M - 2] and L >= 3N
// keeps the cyclic convolution free of wrap-around.  The tables (twiddles of length L, chirp,
// and FFT_L(c) / L) are computed on the host in FP64 (plan.cpp).
//
// Output convention as the power-of-two sweeps: unnormalised, 2 X_k per transform, so the z
// pass's factor 1/(4 M^2) normalises the four transforms of a solve (x and y, forward and
// inverse; the z direction is the tridiagonal solve of z_tri.hip).
//
// Layout: a block loads a tile of 16 lines (runs of 8 FP64 = 128 bytes along y) into LDS,
// each wavefront transforms line pairs with G lanes per pair (L/8 up to 64 lanes), the complex
// FFT exchanging through a padded buffer per pair, and the block stores the tile.
#include "dst_line.h"

namespace dpm {

namespace {

template <int LOGL>
struct BCfg {
  static constexpr int L = 1 << LOGL;
  static constexpr int G = L / 8 < 64 ? L / 8 : 64;  // lanes per line pair
  static constexpr int V = L / G;                     // complex values per lane
  static constexpr int PW = 64 / G;                   // pairs per wavefront at a time
  static constexpr int WAVES = 2;
  static constexpr int T = 64 * WAVES;
  static constexpr int W = LOGL >= 11 ? 8 : 16;       // lines per tile
  static constexpr int NMAX = L / 3;                  // longest line (L >= 3N)
  static constexpr int PITCH = NMAX + 2 + ((NMAX + 2) % 2 == 0 ? 1 : 0);  // odd: no bank conflicts
  static constexpr int BUF = L + L / 8;               // padded FFT buffer (complex)
};

// One Bluestein transform of the pair held in a[] (a[s] = x at position p = g + G s, j = p + 1):
// on return the lane's outputs k = 1 + g + G s (k <= N) are o1[s] = 2 X1_k, o2[s] = 2 X2_k.
template <int LOGL>
__device__ __forceinline__ void blue_transform(C2<double>* a, int g, C2<double>* buf, int N,
                                               int M, const C2<double>* tw,
                                               const C2<double>* wch, const C2<double>* chf,
                                               double* o1, double* o2) {
  using B = BCfg<LOGL>;
  constexpr int L = B::L, V = B::V, G = B::G;
  fft_stages<double, L, V, 1>(a, g, buf, tw);
  // spectrum times the chirp filter's (scaled by 1/L), conjugated: the inverse FFT as a forward
  // one of the conjugate
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = g + s * G;
    const C2<double> A = buf[pad8(k)];
    const C2<double> f = chf[k];
    const C2<double> P = cmul(A, f);
    a[s] = C2<double>{P.x, -P.y};
  }
  wave_sync();
  fft_stages<double, L, V, 1>(a, g, buf, tw);
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = 1 + g + s * G;
    if (k <= N) {
      const C2<double> b1 = buf[pad8(k - 1)];
      const C2<double> b2 = buf[pad8(2 * M - 1 - k)];
      const C2<double> w = wch[k];
      // y = conj(b); Y = w y, Y' = w y(2M - k)
      const C2<double> Y = cmul(w, C2<double>{b1.x, -b1.y});
      const C2<double> Yp = cmul(w, C2<double>{b2.x, -b2.y});
      o1[s] = Y.y - Yp.y;     // 2 Im Y1_k
      o2[s] = Yp.x - Y.x;     // 2 Im Y2_k = -(Re Y_k - Re Y_{2M-k})
    }
  }
  wave_sync();  // every read of the buffer done before the next transform writes it
}

template <int LOGL, int AX>
__global__ __launch_bounds__(BCfg<LOGL>::T) void k_dst_blue(PassArgs p, const double* __restrict__ twd,
                                                           const double* __restrict__ wchd,
                                                           const double* __restrict__ chfd, int N,
                                                           int tiles, int nblocks) {
  using B = BCfg<LOGL>;
  constexpr int T = B::T, W = B::W, G = B::G, V = B::V, PW = B::PW, PITCH = B::PITCH;
  __shared__ __align__(16) double tile[W * PITCH];
  __shared__ __align__(16) C2<double> bufs[B::WAVES * PW * B::BUF];

  const int M = N + 1;
  const long long VOL = (long long)N * N * N;
  const int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  const int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  const long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  const long long S_LINE = (AX == AX_X) ? N : 1;
  const long long S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : (long long)N * N);
  const C2<double>* tw = reinterpret_cast<const C2<double>*>(twd);
  const C2<double>* wch = reinterpret_cast<const C2<double>*>(wchd);
  const C2<double>* chf = reinterpret_cast<const C2<double>*>(chfd);

  const int logical = xcd_remap(blockIdx.x, nblocks);
  const int rhs = logical / tiles;
  const int t = logical - rhs * tiles;
  const int row = t / TILES_PER_ROW;
  const int line0 = (t - row * TILES_PER_ROW) * W;
  const int nlines = min(W, LINES_PER_ROW - line0);
  const long long base = (long long)rhs * VOL + (long long)row * S_OUTER + (long long)line0 * S_LINE;
  const int tid = threadIdx.x;
  const double* __restrict__ in = static_cast<const double*>(p.in) + base;
  double* __restrict__ out = static_cast<double*>(p.out) + base;

  // ---- load: x lines are contiguous (consecutive threads along a line); y and z lines are
  //      adjacent in x (consecutive threads across the W lines of one element); lines past the
  //      row's end are zero (they share a transform with a real line)
  const int cnt = W * N;
  for (int e = tid; e < cnt; e += T) {
    int w, j;
    if constexpr (AX == AX_X) { w = e / N; j = e - w * N; }
    else { j = e / W; w = e - j * W; }
    tile[w * PITCH + j + 1] = w < nlines ? in[(long long)w * S_LINE + (long long)j * S_ELEM] : 0.0;
  }
  __syncthreads();

  // ---- transform the line pairs: wavefront wv, pair slot q within it, lane g of the pair
  const int lane = tid & 63, wv = tid >> 6;
  const int g = lane % G, q = lane / G;
  C2<double>* buf = bufs + (wv * PW + q) * B::BUF;
  constexpr int PAIRS = W / 2;
  constexpr int PER_ROUND = B::WAVES * PW;
  for (int pr0 = 0; pr0 < PAIRS; pr0 += PER_ROUND) {
    const int pr = pr0 + wv * PW + q;  // uniform across the G lanes of a pair
    if (pr < PAIRS) {
      double* l1 = tile + (2 * pr) * PITCH;
      double* l2 = l1 + PITCH;
      C2<double> a[V];
      double o1[V], o2[V];
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int j = 1 + g + s * G;
        a[s] = j <= N ? cmul(C2<double>{l1[j], l2[j]}, wch[j]) : C2<double>{0.0, 0.0};
        o1[s] = 0.0;
        o2[s] = 0.0;
      }
      blue_transform<LOGL>(a, g, buf, N, M, tw, wch, chf, o1, o2);
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int k = 1 + g + s * G;
        if (k <= N) {
          l1[k] = o1[s];
          l2[k] = o2[s];
        }
      }
    }
  }
  __syncthreads();

  // ---- store the tile's real lines
  for (int e = tid; e < cnt; e += T) {
    int w, j;
    if constexpr (AX == AX_X) { w = e / N; j = e - w * N; }
    else { j = e / W; w = e - j * W; }
    if (w < nlines) out[(long long)w * S_LINE + (long long)j * S_ELEM] = tile[w * PITCH + j + 1];
  }
}

template <int LOGL>
dpm_status launch_b(int n, AxisKind ax, const PassArgs& a, const Plan* pl, int nrhs,
                    hipStream_t s) {
  using B = BCfg<LOGL>;
  const long long lines_per_row = (ax == AX_X) ? (long long)n * n : n;
  const long long rows = (ax == AX_X) ? 1 : n;
  const long long tiles = rows * ((lines_per_row + B::W - 1) / B::W);
  const long long nb = tiles * nrhs;
  if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
  const dim3 grid((unsigned)nb), block(B::T);
  const int ti = (int)tiles, nbi = (int)nb;
  if (ax == AX_X)
    hipLaunchKernelGGL((k_dst_blue<LOGL, AX_X>), grid, block, 0, s, a, pl->blue_tw,
                       pl->blue_w, pl->blue_ch, n, ti, nbi);
  else
    hipLaunchKernelGGL((k_dst_blue<LOGL, AX_Y>), grid, block, 0, s, a, pl->blue_tw,
                       pl->blue_w, pl->blue_ch, n, ti, nbi);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace

int blue_logl(int n) {
  if (n < 7 || n > kBlueMaxN) return 0;
  int lg = 7;
  while ((1 << lg) < 3 * n) ++lg;
  return lg;
}

bool blue_size_supported(int n) { return !fft_size_supported(n) && blue_logl(n) != 0; }

dpm_status launch_blue_pass(int n, AxisKind ax, bool zpass, const PassArgs& a, const Plan* pl,
                            int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (ax == AX_Z || zpass) { set_error("the z direction is the tridiagonal pass"); return DPM_EINVAL; }
  if (a.cmax != nullptr || a.done != nullptr) {
    set_error("the Bluestein sweeps serve the plain FP64 solve (no refinement)");
    return DPM_EINVAL;
  }
  if (pl->blue_logl == 0 || pl->blue_logl != blue_logl(n)) {
    set_error("no Bluestein tables for n = %d", n);
    return DPM_EINVAL;
  }
  switch (pl->blue_logl) {
    case 7: return launch_b<7>(n, ax, a, pl, nrhs, s);
    case 8: return launch_b<8>(n, ax, a, pl, nrhs, s);
    case 9: return launch_b<9>(n, ax, a, pl, nrhs, s);
    case 10: return launch_b<10>(n, ax, a, pl, nrhs, s);
    case 11: return launch_b<11>(n, ax, a, pl, nrhs, s);
    default: set_error("no Bluestein sweep for n = %d", n); return DPM_EINVAL;
  }
}

}  // namespace dpm
