// Per-axis DST-I sweeps of the auxiliary-problem solve on gfx950.
//
// The AP (sigma I - Lap_h) u = b with zero Dirichlet data is diagonalised by the orthonormal
// DST-I S (S = S^T = S^-1) along each axis: u = S3 D^-1 S3 b, D = sigma + lambda_kx + lambda_ky
// + lambda_kz.  One solve is five sweeps over the volume: forward x, forward y, a fused z sweep
// (forward, eigenvalue scaling, inverse), inverse y, inverse x.
//
// A sweep moves tiles of W lines (W * sizeof(real) = 128 bytes of each row of the tile, so
// every global access is a run of >= 128 contiguous bytes) into LDS.  Two real lines a, b are
// transformed together by one complex FFT of length L = 2(N+1): the odd extensions of the two
// lines form z = y_a + i y_b, and Z = FFT(z) gives DST(a)_k = -Im Z_k / 2 and
// DST(b)_k = Re Z_k / 2 for k = 1..N.  The FFT is a Stockham radix-8 (last stage radix 2 or 4)
// with every thread holding 8 complex values in registers and LDS between stages; twiddles come
// from an FP64-computed table.
//
// The first x sweep of a refinement step computes the FP64 residual b - (sigma - Lap_h) u on the
// fly; the last x sweep can add its result into u (u += c) and reduce max|c|, max|u|.
#include "common.h"

namespace dpm {

namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> mul_minus_i(C2<T> a) { return {a.y, -a.x}; }
template <typename T>
__device__ __forceinline__ C2<T> mul_plus_i(C2<T> a) { return {-a.y, a.x}; }

// In-register DFTs of size 2, 4, 8 with omega = exp(-2 pi i / R).
template <typename T>
__device__ __forceinline__ void dft2(C2<T>& a0, C2<T>& a1) {
  C2<T> t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}
template <typename T>
__device__ __forceinline__ void dft4(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3) {
  C2<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, mul_minus_i(t3));
  a3 = cadd(t1, mul_plus_i(t3));
}
template <typename T>
__device__ __forceinline__ void dft8(C2<T>* a) {
  C2<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  C2<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const T c = (T)0.70710678118654752440;
  o1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};   // * exp(-i pi/4)
  o2 = mul_minus_i(o2);                          // * exp(-i pi/2)
  o3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};  // * exp(-3i pi/4)
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

template <typename T, int LOG2L>
struct Cfg {
  static constexpr int L = 1 << LOG2L;  // complex FFT length
  static constexpr int M = L / 2;       // N + 1
  static constexpr int N = M - 1;       // line length
  static constexpr int TPF = L / 8;     // threads per FFT (8 values each)
  static constexpr int W = (sizeof(T) == 4) ? 32 : (L >= 2048 ? 8 : 16);  // lines per tile
  static constexpr int NF0 = kBlock / TPF;
  static constexpr int NF = (NF0 < W / 2) ? NF0 : W / 2;  // FFTs in flight per block
  static constexpr int ROUNDS = (W / 2 + NF - 1) / NF;
};

// One Stockham stage of radix R at stride NS on the 8 values a thread holds.  On entry a[s]
// is element j + s*TPF; on exit a[s] is output element pos[s].
template <typename T, int L, int R, int NS>
__device__ __forceinline__ void stage(C2<T>* a, int* pos, int j, const C2<T>* __restrict__ tw) {
  constexpr int TPF = L / 8;
  constexpr int Q = 8 / R;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int v = j + q * TPF;
    const int vm = v & (NS - 1);
    C2<T> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      x[r] = a[q + r * Q];
      if (NS > 1 && r > 0) x[r] = cmul(x[r], tw[(r * vm * (L / (NS * R))) & (L - 1)]);
    }
    if constexpr (R == 8) {
      dft8(x);
    } else if constexpr (R == 4) {
      dft4(x[0], x[1], x[2], x[3]);
    } else {
      dft2(x[0], x[1]);
    }
    const int base = (v - vm) * R + vm;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      a[q + r * Q] = x[r];
      pos[q + r * Q] = base + r * NS;
    }
  }
}

template <int L, int NS>
constexpr int radix_at() {
  return (NS * 8 <= L) ? 8 : L / NS;
}

// Runs the stages from stride NS to the end.  The values for the stage at NS are in a[]
// (element j + s*TPF).  Intermediate results go through buf (this FFT's slot of L values).
// All threads of the block call this (barriers inside); `act` gates the arithmetic.
template <typename T, int L, int NS>
__device__ __forceinline__ void run_stages(C2<T>* a, int* pos, int j, bool act, C2<T>* buf,
                                           const C2<T>* __restrict__ tw) {
  constexpr int R = radix_at<L, NS>();
  constexpr int TPF = L / 8;
  if (act) stage<T, L, R, NS>(a, pos, j, tw);
  if constexpr (NS * R < L) {
    if (act) {
#pragma unroll
      for (int s = 0; s < 8; ++s) buf[pos[s]] = a[s];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int s = 0; s < 8; ++s) a[s] = buf[j + s * TPF];
    }
    __syncthreads();
    run_stages<T, L, NS * R>(a, pos, j, act, buf, tw);
  }
}

// Odd extension of tile line `ln` (length N, pitch N) at index i of the length-2M sequence.
template <typename T, int M>
__device__ __forceinline__ T odd_ext(const T* __restrict__ line, int i) {
  if (i == 0 || i == M) return (T)0;
  if (i < M) return line[i - 1];
  return -line[2 * M - i - 1];
}

template <typename T, int LOG2L, int AX, bool ZPASS, int IN, int OUT>
__global__ __launch_bounds__(kBlock) void k_dst_pass(PassArgs p) {
  using K = Cfg<T, LOG2L>;
  constexpr int L = K::L, M = K::M, N = K::N, TPF = K::TPF, W = K::W, NF = K::NF;
  constexpr long long VOL = (long long)N * N * N;
  // geometry of the tiles: X lines are rows (contiguous), Y/Z lines are columns of W x-values
  constexpr int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  constexpr int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  constexpr long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  constexpr long long S_LINE = (AX == AX_X) ? N : 1;
  constexpr long long S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : (long long)N * N);

  __shared__ T tile[W * N];
  __shared__ C2<T> fbuf[NF * L];
  __shared__ unsigned long long red[2][kBlock / 64];

  const int rhs = blockIdx.y;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;  // converged: uniform exit

  const int t = blockIdx.x;
  const int row = t / TILES_PER_ROW;
  const int ti = t - row * TILES_PER_ROW;
  const int line0 = ti * W;
  const int nlines = min(W, LINES_PER_ROW - line0);
  const long long base = (long long)rhs * VOL + (long long)row * S_OUTER + (long long)line0 * S_LINE;
  const int tid = threadIdx.x;

  // ------------------------------------------------------------------ load the tile
  if constexpr (AX == AX_X) {
    const int cnt = nlines * N;
    for (int e = tid; e < cnt; e += kBlock) {
      const long long g = base + e;
      T v;
      if constexpr (IN == IN_RESID) {
        const int w = e / N;
        const int x = e - w * N;
        const int ln = line0 + w;
        const int z = ln / N;
        const int y = ln - z * N;
        const double* __restrict__ u = p.u;
        const double uc = u[g];
        double nb = 0.0;
        if (x > 0) nb += u[g - 1];
        if (x < N - 1) nb += u[g + 1];
        if (y > 0) nb += u[g - N];
        if (y < N - 1) nb += u[g + N];
        if (z > 0) nb += u[g - (long long)N * N];
        if (z < N - 1) nb += u[g + (long long)N * N];
        const double r = p.b[g] - (p.sigma + 6.0 * p.inv_h2) * uc + p.inv_h2 * nb;
        v = (T)r;
      } else if constexpr (IN == IN_F64) {
        v = (T)(static_cast<const double*>(p.in)[g]);
      } else {
        v = static_cast<const T*>(p.in)[g];
      }
      tile[e] = v;  // (w, x) at w*N + x
    }
  } else {
    const int cnt = N * W;
    for (int e = tid; e < cnt; e += kBlock) {
      const int j = e / W;        // W is a power of two
      const int w = e - j * W;
      if (w < nlines) {
        const long long g = base + w + (long long)j * S_ELEM;
        T v;
        if constexpr (IN == IN_F64) {
          v = (T)(static_cast<const double*>(p.in)[g]);
        } else {
          v = static_cast<const T*>(p.in)[g];
        }
        tile[w * N + j] = v;
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ transform line pairs
  const C2<T>* __restrict__ tw = static_cast<const C2<T>*>(p.tw);
  const int f = tid / TPF;
  const int j = tid - f * TPF;
  C2<T>* buf = fbuf + (f < NF ? f : 0) * L;
  const T c1 = (T)(1.0 / sqrt(2.0 * (double)M));  // orthonormal scale of one DST-I

#pragma unroll 1
  for (int round = 0; round < K::ROUNDS; ++round) {
    const int pair = round * NF + f;
    const int la = 2 * pair;
    const int lb = la + 1;
    const bool act = (f < NF) && (la < nlines);
    const bool hasb = lb < nlines;
    const T* linea = tile + la * N;
    const T* lineb = tile + (hasb ? lb : la) * N;
    C2<T> a[8];
    int pos[8];
    if (act) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int i = j + s * TPF;
        a[s].x = odd_ext<T, M>(linea, i);
        a[s].y = hasb ? odd_ext<T, M>(lineb, i) : (T)0;
      }
    }
    __syncthreads();  // every line of this round read before any write back into the tile
    run_stages<T, L, 1>(a, pos, j, act, buf, tw);

    if constexpr (ZPASS) {
      // scale by 1/(sigma + lambda_kx + lambda_ky + lambda_kz) and restart from the odd
      // extension of the scaled coefficients (S is its own inverse)
      const int kx_a = line0 + la;      // x index of line a (0-based)
      const int kx_b = line0 + lb;
      const int ky = row;               // y index (0-based)
      const double base_a = act ? p.sigma + p.inv_h2 * (p.lam_hat[kx_a] + p.lam_hat[ky]) : 1.0;
      const double base_b = (act && hasb) ? p.sigma + p.inv_h2 * (p.lam_hat[kx_b] + p.lam_hat[ky]) : 1.0;
      if (act) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = pos[s];
          if (k == 0 || k == M) {
            buf[k] = {(T)0, (T)0};
          } else if (k < M) {
            const double lz = p.inv_h2 * p.lam_hat[k - 1];
            const T da = (T)(1.0 / (base_a + lz));
            const T db = (T)(1.0 / (base_b + lz));
            C2<T> w;
            w.x = -a[s].y * c1 * da;
            w.y = a[s].x * c1 * db;
            buf[k] = w;
            buf[2 * M - k] = {-w.x, -w.y};
          }
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int s = 0; s < 8; ++s) a[s] = buf[j + s * TPF];
      }
      __syncthreads();
      run_stages<T, L, 1>(a, pos, j, act, buf, tw);
    }

    // extract DST coefficients k = 1..N of both lines back into the tile
    if (act) {
      T* wa = tile + la * N;
      T* wb = tile + lb * N;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = pos[s];
        if (k >= 1 && k < M) {
          wa[k - 1] = -a[s].y * c1;
          if (hasb) wb[k - 1] = a[s].x * c1;
        }
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ store the tile
  double cm = 0.0, um = 0.0;
  if constexpr (AX == AX_X) {
    const int cnt = nlines * N;
    for (int e = tid; e < cnt; e += kBlock) {
      const long long g = base + e;
      const T v = tile[e];
      if constexpr (OUT == OUT_UPD) {
        double* uo = static_cast<double*>(p.out);
        const double nu = uo[g] + (double)v;
        uo[g] = nu;
        cm = fmax(cm, fabs((double)v));
        um = fmax(um, fabs(nu));
      } else if constexpr (OUT == OUT_F64) {
        static_cast<double*>(p.out)[g] = (double)v;
        cm = fmax(cm, fabs((double)v));
      } else {
        static_cast<T*>(p.out)[g] = v;
        if (p.cmax != nullptr) cm = fmax(cm, fabs((double)v));
      }
    }
  } else {
    const int cnt = N * W;
    for (int e = tid; e < cnt; e += kBlock) {
      const int j2 = e / W;
      const int w = e - j2 * W;
      if (w < nlines) {
        const long long g = base + w + (long long)j2 * S_ELEM;
        static_cast<T*>(p.out)[g] = tile[w * N + j2];
      }
    }
  }

  if constexpr (AX == AX_X) {
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

template <typename T, int LOG2L>
dpm_status launch_t(AxisKind ax, bool zpass, InKind in, OutKind out, const PassArgs& a,
                    int nrhs, hipStream_t s) {
  using K = Cfg<T, LOG2L>;
  constexpr int N = K::N, W = K::W;
  const int lines_per_row = (ax == AX_X) ? N * N : N;
  const int rows = (ax == AX_X) ? 1 : N;
  const int tiles = rows * ((lines_per_row + W - 1) / W);
  dim3 grid(tiles, nrhs), block(kBlock);
  if (ax == AX_X) {
    if (zpass) { set_error("z sweep requested on the x axis"); return DPM_EINVAL; }
    if (in == IN_WS && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_X, false, IN_WS, OUT_WS>), grid, block, 0, s, a);
    else if (in == IN_F64 && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_X, false, IN_F64, OUT_WS>), grid, block, 0, s, a);
    else if (in == IN_RESID && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_X, false, IN_RESID, OUT_WS>), grid, block, 0, s, a);
    else if (in == IN_WS && out == OUT_F64) hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_X, false, IN_WS, OUT_F64>), grid, block, 0, s, a);
    else if (in == IN_WS && out == OUT_UPD) hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_X, false, IN_WS, OUT_UPD>), grid, block, 0, s, a);
    else { set_error("unsupported x sweep kind (%d,%d)", (int)in, (int)out); return DPM_EINVAL; }
  } else if (ax == AX_Y) {
    if (zpass || in != IN_WS || out != OUT_WS) { set_error("unsupported y sweep kind"); return DPM_EINVAL; }
    hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_Y, false, IN_WS, OUT_WS>), grid, block, 0, s, a);
  } else {
    if (!zpass || in != IN_WS || out != OUT_WS) { set_error("unsupported z sweep kind"); return DPM_EINVAL; }
    hipLaunchKernelGGL((k_dst_pass<T, LOG2L, AX_Z, true, IN_WS, OUT_WS>), grid, block, 0, s, a);
  }
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

template <typename T>
dpm_status launch_size(int n, AxisKind ax, bool zpass, InKind in, OutKind out, const PassArgs& a,
                       int nrhs, hipStream_t s) {
  switch (n) {
    case 7: return launch_t<T, 4>(ax, zpass, in, out, a, nrhs, s);
    case 15: return launch_t<T, 5>(ax, zpass, in, out, a, nrhs, s);
    case 31: return launch_t<T, 6>(ax, zpass, in, out, a, nrhs, s);
    case 63: return launch_t<T, 7>(ax, zpass, in, out, a, nrhs, s);
    case 127: return launch_t<T, 8>(ax, zpass, in, out, a, nrhs, s);
    case 255: return launch_t<T, 9>(ax, zpass, in, out, a, nrhs, s);
    case 511: return launch_t<T, 10>(ax, zpass, in, out, a, nrhs, s);
    case 1023: return launch_t<T, 11>(ax, zpass, in, out, a, nrhs, s);
    default: set_error("no FFT sweep for n = %d", n); return DPM_EINVAL;
  }
}

}  // namespace

dpm_status launch_dst_pass(int real_bytes, int n, AxisKind ax, bool zpass, InKind in,
                           OutKind out, const PassArgs& a, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return DPM_OK;
  if (nrhs > 65535) { set_error("too many right-hand sides in one launch"); return DPM_EINVAL; }
  if (real_bytes == 4) return launch_size<float>(n, ax, zpass, in, out, a, nrhs, s);
  // FP64 transforms: FP64 input/output is the native type
  if (in == IN_F64) in = IN_WS;
  if (out == OUT_F64) {
    // storing FP64 from an FP64 tile: same as a plain store, keep the max tracking
    return launch_size<double>(n, ax, zpass, in, OUT_F64, a, nrhs, s);
  }
  return launch_size<double>(n, ax, zpass, in, out, a, nrhs, s);
}

}  // namespace dpm
