// Per-axis DST-I sweeps of the auxiliary-problem solve on gfx950.
//
// The AP (sigma I - Lap_h) u = b with zero Dirichlet data is diagonalised by the orthonormal
// DST-I S (S = S^T = S^-1) along each axis: u = S3 D^-1 S3 b, D = sigma + lambda_kx + lambda_ky
// + lambda_kz.  One solve is five sweeps over the volume: forward x, forward y, a fused z sweep
// (forward, eigenvalue scaling, inverse), inverse y, inverse x.
//
// Sweep layout.  A block moves a tile of W whole lines (W * sizeof(real) = 128 bytes of every
// row of the tile, so each global access is a run of 128 contiguous bytes) into LDS with a
// padded pitch per line, transforms every line in place in its own LDS slot and
// writes the tile back.  Line transforms are wave-local: the G threads of a line sit in one
// wavefront and synchronise with wavefront barriers only; the two block barriers per tile
// separate the cooperative load, the transforms and the store.
//
// Line transform (DST-I of length N = M - 1, M a power of two), through a real DFT of length M:
//   y_j = sin(pi j/M)(x_j + x_{M-j}) + (x_j - x_{M-j})/2,  y_0 = 0,  F = DFT_M(y);
//   then X_2k = -Im F_k and X_2k+1 = X_2k-1 + Re F_k (X_1 = Re F_0 / 2): the odd outputs are a
//   prefix sum, evaluated as a tree scan across the threads of the line.
// The real DFT is a complex FFT of length H = M/2 on w_q = y_2q + i y_2q+1 (Stockham radix-8,
// last stage radix 2 or 4, 8 complex values per thread) followed by the even/odd split
// F_k = (W_k + conj W_{H-k})/2 - i e^{-2 pi i k/M} (W_k - conj W_{H-k})/2.
// Sines and twiddles come from one FP64-computed table held in LDS.
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

// Wavefront-scope barrier for LDS exchanges among the threads of one line.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// Smallest even LDS pitch (reals) that holds a line's x_0..x_M and its padded FFT buffer and
// is congruent to +-2 modulo 32, so the W lines of a strided load hit distinct banks.
constexpr int pitch_for(int M) {
  const int H = M / 2;
  int need = 2 * ((H - 1) + (H - 1) / 8) + 2;
  if (need < M + 1) need = M + 1;
  int p = need + (need & 1);
  while (p % 32 != 2 && p % 32 != 30) p += 2;
  return p;
}

template <typename T, int LOGM>
struct Cfg {
  static constexpr int M = 1 << LOGM;   // N + 1
  static constexpr int N = M - 1;       // line length
  static constexpr int H = M / 2;       // complex FFT length
  static constexpr int V = H >= 8 ? 8 : H;  // complex values per thread
  static constexpr int G = H / V;       // threads per line (divides 64)
  static constexpr int W = (sizeof(T) == 4 ? 32 : 16) / (M >= 1024 ? 2 : 1);  // lines per tile
  // LDS pitch of a line: room for the padded FFT buffer (H + H/8 complex), even so that a
  // line starts on a complex boundary, and not a multiple of the bank count
  static constexpr int P = pitch_for(M);
  static constexpr int LPR = kBlock / G;              // lines per round
  static constexpr int ROUNDS = (W + LPR - 1) / LPR;
};

// Padded position of complex element p in a line's FFT buffer: one pad slot every 8 elements
// keeps the radix-8 stage writes (stride 8) and the post-processing reads conflict-free.
__device__ __forceinline__ int pad8(int p) { return p + (p >> 3); }

template <int H, int NS>
constexpr int radix_at() {
  return (NS * 8 <= H) ? 8 : H / NS;
}

// One Stockham stage of radix R at stride NS over an FFT of length H with V values per
// thread.  On entry a[s] is element g + s*G; on exit a[s] is output element pos[s].
// tw: e^{-2 pi i e/H}, e < H.
template <typename T, int H, int V, int R, int NS>
__device__ __forceinline__ void stage(C2<T>* a, int* pos, int g, const C2<T>* tw) {
  constexpr int G = H / V;
  constexpr int Q = V / R;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int v = g + q * G;
    const int vm = v & (NS - 1);
    C2<T> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      x[r] = a[q + r * Q];
      if (NS > 1 && r > 0) x[r] = cmul(x[r], tw[(r * vm * (H / (NS * R))) & (H - 1)]);
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

// Stages from stride NS to the end, exchanging through `buf` (the line's own slot, padded
// positions).  On return the natural-order result is in buf[pad8(k)] behind a wave barrier.
template <typename T, int H, int V, int NS>
__device__ __forceinline__ void fft_stages(C2<T>* a, int g, C2<T>* buf, const C2<T>* tw) {
  constexpr int R = radix_at<H, NS>();
  constexpr int G = H / V;
  int pos[V];
  stage<T, H, V, R, NS>(a, pos, g, tw);
#pragma unroll
  for (int s = 0; s < V; ++s) buf[pad8(pos[s])] = a[s];
  wave_sync();
  if constexpr (NS * R < H) {
#pragma unroll
    for (int s = 0; s < V; ++s) a[s] = buf[pad8(g + s * G)];
    wave_sync();
    fft_stages<T, H, V, NS * R>(a, g, buf, tw);
  }
}

// Inclusive prefix sum across the G threads of a line (G divides 64; groups are aligned).
// Within a 16-lane DPP row the shifts are row_shr moves; wider groups use lane shuffles.
template <int N>
__device__ __forceinline__ double dpp_shr(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x110 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x110 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int N>
__device__ __forceinline__ float dpp_shr(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + N, 0xF, 0xF, false));
}
template <typename T, int G>
__device__ __forceinline__ T group_scan(T v, int g) {
  if constexpr (G == 16) {
    // the group is exactly one DPP row: shifted-in lanes read 0, no guard needed
    v += dpp_shr<1>(v);
    v += dpp_shr<2>(v);
    v += dpp_shr<4>(v);
    v += dpp_shr<8>(v);
  } else if constexpr (G < 16) {
    if constexpr (G > 1) { const T t = dpp_shr<1>(v); if (g >= 1) v += t; }
    if constexpr (G > 2) { const T t = dpp_shr<2>(v); if (g >= 2) v += t; }
    if constexpr (G > 4) { const T t = dpp_shr<4>(v); if (g >= 4) v += t; }
    if constexpr (G > 8) { const T t = dpp_shr<8>(v); if (g >= 8) v += t; }
  } else {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const T o = __shfl_up(v, off, G);
      if (g >= off) v += o;
    }
  }
  return v;
}

// In-place DST-I of one line by the G threads g = 0..G-1 of the line, unnormalised: on exit
// line[i] = 2 X_i with X_i = sum_j x_j sin(pi i j/M) (the orthonormal transform is
// sqrt(2/M) X; the factors of all six transforms of a solve are applied once, in the z sweep).
// Slot layout (P reals): x_j at line[j], j = 1..N, line[0] = 0, and again line[0] = 0 on exit.  The slot doubles as the
// padded FFT buffer (pad8 positions).  Thread g owns the strided elements g + s*G, so that every
// LDS access of a stage touches consecutive positions.
// tab: [ sin(pi j/M), j < M | e^{-2 pi i e/H}, e < H | e^{-2 pi i k/M}, k < H ].
template <typename T, int LOGM>
__device__ __forceinline__ void dst1_line(T* line, int g, const T* tab) {
  using K = Cfg<T, LOGM>;
  constexpr int M = K::M, H = K::H, V = K::V, G = K::G;
  C2<T>* buf = reinterpret_cast<C2<T>*>(line);
  const T* ts = tab;
  const C2<T>* tw = reinterpret_cast<const C2<T>*>(tab + M);
  const C2<T>* tp = reinterpret_cast<const C2<T>*>(tab + 2 * M);
  // ---- pre-processing into the first stage's registers: element q = g + s*G holds
  //      y_2q + i y_2q+1 with y_j = sin(pi j/M)(x_j + x_{M-j}) + (x_j - x_{M-j})/2, y_0 = 0
  C2<T> a[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int q = g + s * G;
    const C2<T> xa = buf[q];                       // (x_2q, x_2q+1)
    const C2<T> sn = reinterpret_cast<const C2<T>*>(ts)[q];  // (sin(pi 2q/M), sin(pi (2q+1)/M))
    const T xb0 = q > 0 ? line[M - 2 * q] : (T)0;  // x_{M-2q}
    const T xb1 = line[M - 2 * q - 1];             // x_{M-2q-1}
    a[s].x = q > 0 ? sn.x * (xa.x + xb0) + (T)0.5 * (xa.x - xb0) : (T)0;
    a[s].y = sn.y * (xa.y + xb1) + (T)0.5 * (xa.y - xb1);
  }
  wave_sync();  // all reads of x done before the slot is overwritten
  fft_stages<T, H, V, 1>(a, g, buf, tw);
  // ---- post-processing: F_k = E_k + e^{-2 pi i k/M} O_k for k = g + s*G
  T re[V], im[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = g + s * G;
    const C2<T> A = buf[pad8(k)];
    const C2<T> Bc = buf[pad8((H - k) & (H - 1))];
    const C2<T> B = {Bc.x, -Bc.y};
    const C2<T> E = {A.x + B.x, A.y + B.y};  // 2 E_k
    const C2<T> D = {A.x - B.x, A.y - B.y};  // 2 i O_k
    const C2<T> O = {D.y, -D.x};             // -i D = 2 O_k
    const C2<T> F = cadd(E, cmul(tp[k], O));  // 2 F_k
    re[s] = F.x;
    im[s] = F.y;
  }
  // ---- X_{2k+1} = sum_{k' <= k} Re F_k' - Re F_0 / 2 (here all doubled): prefix in k = g + s*G order, i.e. a
  //      scan across the line's threads for each s plus the totals of the rows before it
  const T f0 = __shfl(re[0], 0, G);  // Re F_0 (element k = 0: s = 0, g = 0)
  T carry = -(T)0.5 * f0;
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const T incl = group_scan<T, G>(re[s], g);
    const T tot = __shfl(incl, G - 1, G);
    re[s] = carry + incl;
    carry += tot;
  }
  wave_sync();  // all reads of the FFT result done before X overwrites the slot
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = g + s * G;
    C2<T> o;
    o.x = k > 0 ? -im[s] : (T)0;  // 2 X_2k   (line[0] = 0 for k = 0)
    o.y = re[s];                  // 2 X_2k+1
    buf[k] = o;
  }
  wave_sync();
}



// ---------------------------------------------------------------------------------------
// Line transform with explicit LDS addressing, for G a multiple of 8 (N >= 127).  Every
// position a thread touches is a per-thread part a plus a compile-time part c, where c is a
// multiple of 8 or a + c has c's low three bits on top of a multiple of 8; in both cases
// pad8(a + c) = pad8(a) + c + c/8, so each LDS access is a per-thread base plus an immediate.

// One Stockham stage (radix R, stride NS) writing its outputs to their padded positions.
// On entry a[s] holds element g + s*G.  KEEP (the last stage): the outputs also stay in a[],
// output r of butterfly q in slot q + r*Q, which is the lane's own element g + (q + r*Q)*G.
template <typename T, int H, int V, int R, int NS, bool KEEP>
__device__ __forceinline__ void stage_w(C2<T>* a, int g, C2<T>* buf, const C2<T>* tw) {
  constexpr int G = H / V;
  constexpr int Q = V / R;
  constexpr int KT = H / (NS * R);  // twiddle index stride
  static_assert(G % 8 == 0, "explicit addressing needs G % 8 == 0");
  int a_thr, vmk;
  if constexpr (NS <= G) {
    const int gm = g & (NS - 1);
    a_thr = (g - gm) * R + gm;  // (v - vm) R + vm with vm = g mod NS
    vmk = gm * KT;
  } else {
    a_thr = g;                  // vm = g + (q G mod NS)
    vmk = g * KT;
  }
  C2<T>* wb = buf + (a_thr + (a_thr >> 3));
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int cq = NS <= G ? 0 : (q * G) % NS;
    C2<T> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = a[q + r * Q];
    if constexpr (NS > 1 && sizeof(T) == 4) {
      // FP32: twiddles as read from the table (each rounded once from FP64)
#pragma unroll
      for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[r * (vmk + cq * KT)]);
    } else if constexpr (NS > 1) {
      // FP64: twiddle w^r for r < R from one table read: w^2 = w w, w^3 = w^2 w, w^4 = w^2 w^2,
      // ... (at most four roundings deep, a few ulp)
      C2<T> wr[R];
      wr[1] = tw[vmk + cq * KT];
      if constexpr (R > 2) {
        wr[2] = cmul(wr[1], wr[1]);
        wr[3] = cmul(wr[2], wr[1]);
      }
      if constexpr (R > 4) {
        wr[4] = cmul(wr[2], wr[2]);
        wr[5] = cmul(wr[4], wr[1]);
        wr[6] = cmul(wr[3], wr[3]);
        wr[7] = cmul(wr[6], wr[1]);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) x[r] = cmul(x[r], wr[r]);
    }
    if constexpr (R == 8) {
      dft8(x);
    } else if constexpr (R == 4) {
      dft4(x[0], x[1], x[2], x[3]);
    } else {
      dft2(x[0], x[1]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = NS <= G ? q * G * R + r * NS : (q * G - cq) * R + cq + r * NS;
      wb[c + c / 8] = x[r];
    }
    if constexpr (KEEP) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[q + r * Q] = x[r];
    }
  }
}

template <typename T, int H, int V, int NS>
__device__ __forceinline__ void fft_stages_w(C2<T>* a, int g, C2<T>* buf, const C2<T>* tw) {
  constexpr int R = radix_at<H, NS>();
  constexpr int G = H / V;
  stage_w<T, H, V, R, NS, (NS * R >= H)>(a, g, buf, tw);
  wave_sync();
  if constexpr (NS * R < H) {
    const C2<T>* rb = buf + (g + (g >> 3));
#pragma unroll
    for (int s = 0; s < V; ++s) a[s] = rb[s * (G + G / 8)];
    wave_sync();
    fft_stages_w<T, H, V, NS * R>(a, g, buf, tw);
  }
}

// Broadcast of lane n of each 16-lane DPP row to the whole row.
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + L, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + L, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int L>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + L, 0xF, 0xF, false));
}
template <typename T, int G>
__device__ __forceinline__ T group_bcast_first(T v) {
  if constexpr (G == 16) return row_bcast<0>(v);
  else return __shfl(v, 0, G);
}
template <typename T, int G>
__device__ __forceinline__ T group_bcast_last(T v) {
  if constexpr (G == 16) return row_bcast<15>(v);
  else return __shfl(v, G - 1, G);
}

// Unnormalised DST-I of one line (as dst1_line) into registers: on exit o[s] = (2 X_2k,
// 2 X_2k+1) for k = g + s*G, and the slot may be overwritten.  FROMREG: the pairs
// (x_2q, x_2q+1), q = g + s*G, are taken from o[] instead of the slot (the slot must still
// hold the line in natural layout for the mirrored reads).
template <typename T, int LOGM, bool FROMREG>
__device__ __forceinline__ void dst1_regs(T* line, int g, const T* tab, const T* gtab, C2<T>* o) {
  using K = Cfg<T, LOGM>;
  constexpr int M = K::M, H = K::H, V = K::V, G = K::G;
  constexpr int G9 = G + G / 8;
  C2<T>* buf = reinterpret_cast<C2<T>*>(line);
  const C2<T>* tw = reinterpret_cast<const C2<T>*>(tab + M);
  const T* lb = line + (M - 2 * g - 2 * (V - 1) * G);  // lb[2 (V-1-s) G] = x_{M-2q}
  const C2<T>* xb = buf + g;
  // E_s = e^{-2 pi i k/M} for the lane's indices k = g + s*G (pre-processing uses q = k):
  // E_0 from the LDS table, E_s = E_0 rho_s with rho_s = e^{-2 pi i s G/M} read uniformly
  // from the global table (scalar loads)
  // (FP64 only; FP32 reads every value from the table, each rounded once from FP64)
  constexpr bool REG = sizeof(T) == 8;
  const C2<T>* gtp = reinterpret_cast<const C2<T>*>(gtab + 2 * M);
  const C2<T>* ltp = reinterpret_cast<const C2<T>*>(tab + 2 * M) + g;
  const C2<T>* lsn = reinterpret_cast<const C2<T>*>(tab) + g;
  C2<T> E[V];
  E[0] = ltp[0];
#pragma unroll
  for (int s = 1; s < V; ++s) E[s] = REG ? cmul(E[0], gtp[s * G]) : ltp[s * G];
  // sin(pi 2q/M) = -Im E, sin(pi (2q+1)/M) = sin(2 pi q/M) cos(pi/M) + cos(2 pi q/M) sin(pi/M)
  const T s1 = gtab[1];          // sin(pi/M)
  const T c1 = gtab[M / 2 - 1];  // cos(pi/M) = sin(pi (M/2 - 1)/M)
  C2<T> a[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const C2<T> xa = FROMREG ? o[s] : xb[s * G];
    const C2<T> snt = REG ? C2<T>{-E[s].y, -E[s].y * c1 + E[s].x * s1} : lsn[s * G];
    const T sn0 = snt.x;
    const T sn1 = snt.y;
    const T xb0 = lb[2 * (V - 1 - s) * G];      // for q = 0: line[M], not used
    const T xb1 = lb[2 * (V - 1 - s) * G - 1];
    const T ax = sn0 * (xa.x + xb0) + (T)0.5 * (xa.x - xb0);
    a[s].x = (s == 0 && g == 0) ? (T)0 : ax;
    a[s].y = sn1 * (xa.y + xb1) + (T)0.5 * (xa.y - xb1);
  }
  wave_sync();
  fft_stages_w<T, H, V, 1>(a, g, buf, tw);
  // F_k = E_k + e^{-2 pi i k/M} O_k.  The lane's own FFT outputs k = g + s*G are still in a[s]
  // (the last stage keeps them); the mirror (H - k) mod H, another lane's, is read from LDS at
  // pad8(G - g) + (V-1-s) G9, except k = 0, whose mirror is 0
  const C2<T>* pm = buf + (g > 0 ? (G - g) + ((G - g) >> 3) : G9);
  const C2<T>* pm0 = g > 0 ? pm + (V - 1) * G9 : buf;
  T re[V], im[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const C2<T> A = a[s];
    const C2<T> Bc = s == 0 ? *pm0 : pm[(V - 1 - s) * G9];
    const C2<T> B = {Bc.x, -Bc.y};
    const C2<T> Ev = {A.x + B.x, A.y + B.y};
    const C2<T> D = {A.x - B.x, A.y - B.y};
    const C2<T> O = {D.y, -D.x};
    const C2<T> F = cadd(Ev, cmul(E[s], O));
    re[s] = F.x;
    im[s] = F.y;
  }
  const T f0 = group_bcast_first<T, G>(re[0]);
  T carry = -(T)0.5 * f0;
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const T incl = group_scan<T, G>(re[s], g);
    const T tot = group_bcast_last<T, G>(incl);
    re[s] = carry + incl;
    carry += tot;
  }
#pragma unroll
  for (int s = 0; s < V; ++s) {
    o[s].x = (s == 0 && g == 0) ? (T)0 : -im[s];
    o[s].y = re[s];
  }
  wave_sync();  // all reads of the FFT result done before the slot is overwritten
}

// 1/d to FP64 accuracy: hardware reciprocal and two Newton steps.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}

// Loads and stores at a uniform base plus a 32-bit byte offset (the global saddr form).  The
// base is passed through readfirstlane so that it stays in scalar registers: the compiler then
// moves a step's base with scalar adds instead of a 64-bit vector add per element.  Callers pass
// pointers that are uniform across the wavefront.
template <typename T>
__device__ __forceinline__ T* sbase(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}
#define DPM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ld(const T* base, unsigned byte_off) {
  const DPM_GLOBAL char* b = (const DPM_GLOBAL char*)sbase(base);
  return *(const DPM_GLOBAL T*)(b + byte_off);
}
template <typename T>
__device__ __forceinline__ void st(T* base, unsigned byte_off, T v) {
  DPM_GLOBAL char* b = (DPM_GLOBAL char*)sbase(base);
  *(DPM_GLOBAL T*)(b + byte_off) = v;
}

// blockIdx -> logical tile such that consecutive logical tiles run on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so neighbouring tiles that share cache lines and
// stencil rows share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// FP64 sweeps at N = 127 and 255 read their tables from global memory (L1/L2 resident) and are
// compiled for 4 waves per SIMD: with at most 38.7 KB of LDS per block, 4 blocks share a CU
// (the fused z sweep, two transforms per line, is bound by LDS latency at 3).  FP32 sweeps and
// N >= 511 (two blocks per CU at most) keep the tables in LDS.
template <typename T, int LOGM, bool ZPASS>
struct ZOcc {
  static constexpr bool gtab = sizeof(T) == 8 && Cfg<T, LOGM>::G % 8 == 0 && LOGM <= 8;
  static constexpr int waves = gtab ? 4 : 1;
};

template <typename T, int LOGM, int AX, bool ZPASS, int IN, int OUT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ZOcc<T, LOGM, ZPASS>::waves)))
void k_dst_pass(PassArgs p, int tiles, int nblocks) {
  using K = Cfg<T, LOGM>;
  constexpr bool GTAB = ZOcc<T, LOGM, ZPASS>::gtab;
  constexpr int M = K::M, N = K::N, G = K::G, W = K::W, P = K::P;
  constexpr long long VOL = (long long)N * N * N;
  constexpr int LINES_PER_ROW = (AX == AX_X) ? N * N : N;
  constexpr int TILES_PER_ROW = (LINES_PER_ROW + W - 1) / W;
  constexpr long long S_OUTER = (AX == AX_X) ? 0 : (AX == AX_Y ? (long long)N * N : N);
  constexpr long long S_LINE = (AX == AX_X) ? N : 1;
  constexpr long long S_ELEM = (AX == AX_X) ? 1 : (AX == AX_Y ? N : (long long)N * N);

  __shared__ __align__(16) T tile[W * P];
  __shared__ __align__(16) T tab[GTAB ? 2 : 3 * M];
  // eigenvalue table of the z sweep: lamt[0] = 0, lamt[i] = lam_hat_i (i = 1..N)
  __shared__ __align__(16) double lamt[ZPASS ? M : 2];
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
    if constexpr (ZPASS) {
      for (int i = tid; i < M; i += kBlock) lamt[i] = i == 0 ? 0.0 : p.lam_hat[i - 1];
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
          const double uc = ld(ub, off), rb = ld(bb, off);
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
  } else {
    // flat mapping: thread owns tile elements e = tid + i*kBlock (x lines, narrow reals)
    const int cnt = nlines * N;
#pragma unroll 1
    for (int c0 = 0; c0 < PER; c0 += CH) {
      T v[CH];
      if constexpr (IN == IN_RESID) {
#pragma unroll
        for (int i0 = 0; i0 < CH; i0 += 4) {
          constexpr int K4 = CH < 4 ? CH : 4;
          double rb[K4], uc[K4], nb[K4];
#pragma unroll
          for (int k = 0; k < K4; ++k) {
            const int e = min(tid + (c0 + i0 + k) * kBlock, cnt - 1);
            const int ww = e / N;
            const int x = e - ww * N;
            const int ln = line0 + ww;
            const int z = ln / N;
            const int y = ln - z * N;
            const double* __restrict__ u = p.u + base;
            uc[k] = u[e];
            rb[k] = p.b[base + e];
            double a0 = x > 0 ? u[e - 1] : 0.0;
            double a1 = x < N - 1 ? u[e + 1] : 0.0;
            double a2 = y > 0 ? u[e - N] : 0.0;
            double a3 = y < N - 1 ? u[e + N] : 0.0;
            double a4 = z > 0 ? u[e - N * N] : 0.0;
            double a5 = z < N - 1 ? u[e + N * N] : 0.0;
            nb[k] = (a0 + a1) + (a2 + a3) + (a4 + a5);
          }
#pragma unroll
          for (int k = 0; k < K4; ++k)
            v[i0 + k] = (T)(rb[k] - (sig + 6.0 * p.inv_h2) * uc[k] + p.inv_h2 * nb[k]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = min(tid + (c0 + i) * kBlock, cnt - 1);
          if constexpr (IN == IN_F64) v[i] = (T)in_d[e];
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
        if constexpr (ZPASS) {
          // scale X_i by (sqrt(2/M)/2)^6 / (sigma + lambda_x + lambda_y + lambda_z), i = 2k, 2k+1
          const double bxy = sig + p.inv_h2 * (p.lam_hat[line0 + l] + p.lam_hat[row]);
          constexpr double kNorm = 1.0 / (8.0 * (double)M * (double)M * (double)M);
          // (lambda_2k, lambda_2k+1) as one aligned 16-byte read
          const C2<double>* lp = reinterpret_cast<const C2<double>*>(lamt) + g;
#pragma unroll
          for (int s2 = 0; s2 < K::V; ++s2) {
            const C2<double> lv = lp[s2 * G];
            const double d0 = kNorm * recip(bxy + p.inv_h2 * lv.x);
            const double d1 = kNorm * recip(bxy + p.inv_h2 * lv.y);
            o[s2].x = (T)((double)o[s2].x * d0);
            o[s2].y = (T)((double)o[s2].y * d1);
            ob[s2 * G] = o[s2];
          }
          wave_sync();
          dst1_regs<T, LOGM, true>(line, g, ttab, gtab_k, o);
        }
#pragma unroll
        for (int s2 = 0; s2 < K::V; ++s2) ob[s2 * G] = o[s2];
        wave_sync();
      } else if constexpr (ZPASS) {
        // forward DST scaled by 1/(sigma + lambda), then the inverse DST: one code path run
        // twice keeps the register footprint of a single transform
        const double bxy = sig + p.inv_h2 * (p.lam_hat[line0 + l] + p.lam_hat[row]);
        // (sqrt(2/M) / 2)^6: normalisation of the six unnormalised transforms of the solve
        constexpr double kNorm = 1.0 / (8.0 * (double)M * (double)M * (double)M);
#pragma unroll 1
        for (int rep = 0; rep < 2; ++rep) {
          dst1_line<T, LOGM>(line, g, tab);
          if (rep == 0) {
#pragma unroll 4
            for (int i = 1 + g; i <= N; i += G)
              line[i] *= (T)(kNorm / (bxy + p.inv_h2 * p.lam_hat[i - 1]));
            wave_sync();
          }
        }
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
  if (ax == AX_X) {
    if (zpass) { set_error("z sweep requested on the x axis"); return DPM_EINVAL; }
    if (in == IN_WS && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, false, IN_WS, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_F64 && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, false, IN_F64, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_RESID && out == OUT_WS) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, false, IN_RESID, OUT_WS>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_WS && out == OUT_F64) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, false, IN_WS, OUT_F64>), grid, block, 0, s, a, ti, nbi);
    else if (in == IN_WS && out == OUT_UPD) hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_X, false, IN_WS, OUT_UPD>), grid, block, 0, s, a, ti, nbi);
    else { set_error("unsupported x sweep kind (%d,%d)", (int)in, (int)out); return DPM_EINVAL; }
  } else if (ax == AX_Y) {
    if (zpass || in != IN_WS || out != OUT_WS) { set_error("unsupported y sweep kind"); return DPM_EINVAL; }
    hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_Y, false, IN_WS, OUT_WS>), grid, block, 0, s, a, ti, nbi);
  } else {
    if (!zpass || in != IN_WS || out != OUT_WS) { set_error("unsupported z sweep kind"); return DPM_EINVAL; }
    hipLaunchKernelGGL((k_dst_pass<T, LOGM, AX_Z, true, IN_WS, OUT_WS>), grid, block, 0, s, a, ti, nbi);
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
  if (real_bytes == 4) return launch_size<float>(n, ax, zpass, in, out, a, nrhs, s);
  // FP64 transforms: FP64 input is the native type
  if (in == IN_F64) in = IN_WS;
  return launch_size<double>(n, ax, zpass, in, out, a, nrhs, s);
}

}  // namespace dpm
