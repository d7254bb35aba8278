// Line transforms of the DST-I sweeps (device code shared by the per-axis sweeps of
// dst_fft.hip and the fused plane sweeps of xy_plane.hip).
//
// Line transform (DST-I of length N = M - 1, M a power of two), through a real DFT of length M:
//   y_j = sin(pi j/M)(x_j + x_{M-j}) + (x_j - x_{M-j})/2,  y_0 = 0,  F = DFT_M(y);
//   then X_2k = -Im F_k and X_2k+1 = X_2k-1 + Re F_k (X_1 = Re F_0 / 2): the odd outputs are a
//   prefix sum, evaluated as a tree scan across the threads of the line.
// The real DFT is a complex FFT of length H = M/2 on w_q = y_2q + i y_2q+1 (Stockham radix-8,
// last stage radix 2 or 4, 8 complex values per thread) followed by the even/odd split
// F_k = (W_k + conj W_{H-k})/2 - i e^{-2 pi i k/M} (W_k - conj W_{H-k})/2.
// A line occupies one LDS slot of P reals that doubles as its padded FFT buffer; the G threads
// of a line sit in one wavefront and synchronise with wavefront barriers only.
#pragma once

#include "common.h"

namespace dpm {

namespace {

// threads per block of the per-axis sweeps
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
// sqrt(2/M) X; the factors of the four x and y transforms of a solve are applied once, by the
// z pass).
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
// Lane l's value of v, read into scalar registers (l must be uniform).
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same load with the non-temporal hint: data read once, not to be kept in the caches.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* base, unsigned byte_off) {
  const DPM_GLOBAL char* b = (const DPM_GLOBAL char*)sbase(base);
  return __builtin_nontemporal_load((const DPM_GLOBAL T*)(b + byte_off));
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

}  // namespace

}  // namespace dpm
