// CholeskyQR2 of the boundary matrix (Algorithm "Main Steps", Step 2: the QR behind the
// reduced BEP's least squares, eq BEP_recast), FP64 on blocked kernels.
//
// A (m x n, column-major) = Q R with Q explicit:
//   pass 1: G1 = A^T A, R1 = chol(G1) (G1 = R1^T R1), Q1 = A R1^-1;
//   pass 2: G2 = Q1^T Q1, R2 = chol(G2), Q = Q1 R2^-1, R = R2 R1;
// and the least-squares operator P = R^-1 Q^T (n x m, row-major), so that C = P g.  Pass 1
// alone loses orthogonality like kappa(A)^2 u; pass 2 restores it to O(u) while
// kappa(Q1) stays near 1, i.e. while G2 stays near the identity.  The driver therefore checks
// that neither Cholesky broke down, that every diagonal entry of R2 lies within 0.05 of 1
// (kappa(A)^2 u well below 1) and that min / max |R_ii| >= 1e-5 (a well-conditioned matrix);
// otherwise A is still intact and the Householder QR takes over.
//
// Work is BLAS-3 shaped: two Gram products (m n^2 flops each, upper tiles, row chunks reduced
// in a fixed order), three products of a triangular n x n factor with an n x m row-major
// matrix (A, Q1 and Q stored column-major are exactly such matrices), and small blocked
// factorisations of n x n matrices in 32 x 32 tiles (left-looking Cholesky with the inverse of
// the factor built alongside, one launch per tile panel).
#include <cmath>

#include "bep.h"

namespace dpm {

namespace {

constexpr int kT = 32;    // tile of the n x n factors
constexpr int kST = 64;   // output tile of the Gram product

// Gp[chunk] (n x n row-major) holds the partial Gram X^T X over the chunk's rows for the tile
// pairs (ta <= tb) of 64 x 64; X is m x n column-major.  Thread (tx, ty) owns the 4 x 4 outputs
// (a0 + 4 tx + u, b0 + 4 ty + v), read from LDS as 16-byte pairs; rows are staged through LDS
// 32 at a time.
constexpr int kSP = kST + 4;  // LDS row pitch of the staged tiles (16-byte aligned rows)
__global__ __launch_bounds__(256) void k_syrk_part(const double* __restrict__ X, int m, int n,
                                                   int rc, double* __restrict__ Gp) {
  __shared__ __align__(16) double xa[kT][kSP], xb[kT][kSP];  // [row][column]
  const int nt = (n + kST - 1) / kST;
  int tile = blockIdx.x, ta = 0;
  while (tile >= nt - ta) { tile -= nt - ta; ++ta; }
  const int tb = ta + tile;
  const int a0 = ta * kST, b0 = tb * kST;
  const int i_lo = blockIdx.y * rc, i_hi = min(m, i_lo + rc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  const int lr = threadIdx.x & 31, lc = threadIdx.x >> 5;  // loader: row lr, columns lc + 8q
  for (int i0 = i_lo; i0 < i_hi; i0 += kT) {
    const int i = i0 + lr;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ca = a0 + lc + 8 * q, cb = b0 + lc + 8 * q;
      xa[lr][lc + 8 * q] = (i < i_hi && ca < n) ? X[(long long)ca * m + i] : 0.0;
      xb[lr][lc + 8 * q] = (i < i_hi && cb < n) ? X[(long long)cb * m + i] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kT; ++r) {
      const double2 a01 = *reinterpret_cast<const double2*>(&xa[r][4 * tx]);
      const double2 a23 = *reinterpret_cast<const double2*>(&xa[r][4 * tx + 2]);
      const double2 b01 = *reinterpret_cast<const double2*>(&xb[r][4 * ty]);
      const double2 b23 = *reinterpret_cast<const double2*>(&xb[r][4 * ty + 2]);
      const double av[4] = {a01.x, a01.y, a23.x, a23.y};
      const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
    }
    __syncthreads();
  }
  double* g = Gp + (long long)blockIdx.y * n * n;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = a0 + 4 * tx + u, cb = b0 + 4 * ty + v;
      if (ra < n && cb < n) g[(long long)ra * n + cb] = acc[u][v];
    }
}

// G[a][b] = G[b][a] = sum over chunks of Gp[chunk][a][b] (a <= b, written by k_syrk_part for
// a <= b within the upper tile pairs): one wavefront per entry, chunks in a fixed order.
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ Gp, int nchunk,
                                                     int n, double* __restrict__ G) {
  const long long e = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= (long long)n * n) return;  // uniform across the wavefront
  const int ra = (int)(e / n), cb = (int)(e - (long long)ra * n);
  if (ra > cb) return;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += Gp[(long long)c * n * n + e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    G[e] = s;
    G[(long long)cb * n + ra] = s;
  }
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned long long)(unsigned)lo);
}

// Lanes 0..31 of one wavefront (lane c = column c in registers, the other lanes inactive):
// the upper Cholesky factor U of the 32 x 32 SPD matrix a (a = U^T U; written back with zeros
// below the diagonal) and ui = U^-1.  Row k of U reaches every lane by readlane, so neither
// step needs a barrier.  A pivot <= 0 or not finite sets *bad and is replaced by 1.
__device__ __forceinline__ void wave_chol_inv(double (*a)[kT + 1], double (*ui)[kT + 1],
                                              int* bad) {
  const int c = threadIdx.x & 63;
  double col[kT];
#pragma unroll
  for (int r = 0; r < kT; ++r) col[r] = a[r][c];
#pragma unroll
  for (int k = 0; k < kT; ++k) {
    double d = readlane_d(col[k], k);
    if (!(d > 0.0) || !isfinite(d)) {  // uniform: d is a scalar
      if (c == 0) *bad = 1;
      d = 1.0;
    }
    const double u = sqrt(d), iu = 1.0 / u;
    col[k] = c == k ? u : (c > k ? col[k] * iu : 0.0);  // row k of U
#pragma unroll
    for (int i = k + 1; i < kT; ++i) {
      const double uki = readlane_d(col[k], i);
      if (c >= i) col[i] -= uki * col[k];
    }
  }
#pragma unroll
  for (int r = 0; r < kT; ++r) a[r][c] = col[r];
  // column c of U^-1 from the bottom: x_r = (delta_rc - sum_{k > r} U_rk x_k) / U_rr
  double x[kT];
#pragma unroll
  for (int r = kT - 1; r >= 0; --r) {
    double acc = r == c ? 1.0 : 0.0;
#pragma unroll
    for (int k = r + 1; k < kT; ++k) acc -= readlane_d(col[r], k) * x[k];
    x[r] = acc / readlane_d(col[r], r);
  }
#pragma unroll
  for (int r = 0; r < kT; ++r) ui[r][c] = x[r];
}

// Panel p of the upper Cholesky factor R (G = R^T R) and of X = R^-1 (all n x n row-major),
// left-looking, in one launch of nt + 1 blocks.  Every block forms S_pp = G_pp - sum_{q<p}
// R_qp^T R_qp and factors it, S_pp = U^T U with U^-1, by one wavefront (the same values in the
// same order in every block).  Blocks b < nt - p then write tile row p of R: block j = p + b
// forms S_pj likewise and writes R_pj = U^-T S_pj (R_pp = U).  Blocks b >= nt - p write tile
// column p of X: row tile i = b - (nt - p) gets X_ip = -(sum_{i<=k<p} X_ik R_kp) U^-1 (X_pp =
// U^-1), from tiles of earlier launches.  Padding rows and columns past n act as the identity.
// A pivot <= 0 or not finite sets *bad and is replaced by 1 (the driver then discards the
// result).
constexpr int kCh = 7;  // tiles staged per chunk (2 x 7 tiles: 118 KB of LDS)
__global__ __launch_bounds__(256) void k_chol_panel(const double* __restrict__ G,
                                                    double* __restrict__ R,
                                                    double* __restrict__ X, int n, int p,
                                                    int* __restrict__ bad) {
  __shared__ double sp[kT][kT + 1], sj[kT][kT + 1], ui[kT][kT + 1];
  __shared__ double ta[kCh][kT][kT + 1], tb[kCh][kT][kT + 1];
  const int nt = (n + kT - 1) / kT;
  const bool rblock = (int)blockIdx.x < nt - p;
  const int j = rblock ? p + (int)blockIdx.x : p;           // R: tile column
  const int xi = rblock ? 0 : (int)blockIdx.x - (nt - p);   // X: tile row
  const int r0 = p * kT, c0 = j * kT, i0 = xi * kT;
  const int t = threadIdx.x;
  // accp: S_pp; accj: S_pj (R blocks) or T = sum_{xi <= k < p} X_{xi,k} R_kp (X blocks)
  double accp[4], accj[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + 256 * q, row = e >> 5, col = e & 31;
    const bool rin = r0 + row < n;
    accp[q] = (rin && r0 + col < n) ? G[(long long)(r0 + row) * n + r0 + col] : (row == col ? 1.0 : 0.0);
    accj[q] = (rblock && rin && c0 + col < n) ? G[(long long)(r0 + row) * n + c0 + col] : 0.0;
  }
  // the earlier tile rows q < p, kCh at a time: every load of a chunk is issued before the
  // first store to LDS (one memory latency per chunk).  ta[u] = R_qp; tb[u] = R_qj (R blocks,
  // j > p) or X_{xi,q} (X blocks, q >= xi).
  for (int qb = 0; qb < p; qb += kCh) {
    const int cnt = min(kCh, p - qb);
    double va[kCh][4], vb[kCh][4];
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      const int qt = qb + u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q, row = e >> 5, col = e & 31;
        const int q0 = qt * kT;
        va[u][q] = (u < cnt && r0 + col < n) ? R[(long long)(q0 + row) * n + r0 + col] : 0.0;
        if (rblock)
          vb[u][q] = (u < cnt && j != p && c0 + col < n) ? R[(long long)(q0 + row) * n + c0 + col] : 0.0;
        else
          vb[u][q] = (u < cnt && qt >= xi) ? X[(long long)(i0 + row) * n + q0 + col] : 0.0;
      }
    }
    if (qb > 0) __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int u = 0; u < kCh; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q, row = e >> 5, col = e & 31;
        ta[u][row][col] = va[u][q];
        tb[u][row][col] = vb[u][q];
      }
    __syncthreads();
    for (int u = 0; u < cnt; ++u) {
      const bool tx = !rblock && qb + u >= xi;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q, row = e >> 5, col = e & 31;
        double sp_ = 0.0, sj_ = 0.0;
        if (rblock) {
#pragma unroll 8
          for (int k = 0; k < kT; ++k) {
            sp_ += ta[u][k][row] * ta[u][k][col];
            sj_ += ta[u][k][row] * tb[u][k][col];
          }
          accj[q] -= sj_;
        } else {
#pragma unroll 8
          for (int k = 0; k < kT; ++k) {
            sp_ += ta[u][k][row] * ta[u][k][col];
            sj_ += tb[u][row][k] * ta[u][k][col];
          }
          if (tx) accj[q] += sj_;
        }
        accp[q] -= sp_;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + 256 * q, row = e >> 5, col = e & 31;
    sp[row][col] = accp[q];
    sj[row][col] = accj[q];
  }
  __syncthreads();
  // S_pp = U^T U by one wavefront, with U^-1 in ui
  if (t < kT) wave_chol_inv(sp, ui, bad);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + 256 * q, row = e >> 5, col = e & 31;
    double a = 0.0;
    if (rblock) {
      if (j == p) {
        a = sp[row][col];
      } else {  // R_pj = U^-T S_pj (U^-T lower: terms k <= row)
        for (int k = 0; k <= row; ++k) a += ui[k][row] * sj[k][col];
      }
      if (r0 + row < n && c0 + col < n) R[(long long)(r0 + row) * n + c0 + col] = a;
    } else {
      if (xi == p) {
        a = ui[row][col];
      } else {  // X_{xi,p} = -T U^-1 (U^-1 upper: terms k <= col)
        for (int k = 0; k <= col; ++k) a += sj[row][k] * ui[k][col];
        a = -a;
      }
      if (i0 + row < n && r0 + col < n) X[(long long)(i0 + row) * n + r0 + col] = a;
    }
  }
}

// Out (n x m, row-major) = L In (In n x m row-major), L = R (TRANS false: upper, terms k >= nu)
// or R^T (TRANS true: lower, terms k <= nu) with R n x n row-major upper triangular.  A block
// owns 32 rows nu and 256 columns i (one per thread, 32 accumulators); the L tile sits in LDS
// and each In element, read once per block from a coalesced row, feeds 32 products.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_tri_apply(const double* __restrict__ Rm, int n,
                                                   const double* __restrict__ In, int m,
                                                   double* __restrict__ Out) {
  __shared__ __align__(16) double lt[kT][kT];  // [k][nu]: row k read as 16 pairs (broadcast)
  const int nu0 = blockIdx.y * kT;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int ic = i < m ? i : m - 1;
  double acc[kT];
#pragma unroll
  for (int v = 0; v < kT; ++v) acc[v] = 0.0;
  const int kt_lo = TRANS ? 0 : blockIdx.y;
  const int kt_hi = TRANS ? blockIdx.y : (n + kT - 1) / kT - 1;
  for (int kt = kt_lo; kt <= kt_hi; ++kt) {
    const int k0 = kt * kT;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q, k = e >> 5, v = e & 31;
      const int gn = nu0 + v, gk = k0 + k;
      double l = 0.0;
      if (gn < n && gk < n)
        l = TRANS ? (gk <= gn ? Rm[(long long)gk * n + gn] : 0.0)
                  : (gk >= gn ? Rm[(long long)gn * n + gk] : 0.0);
      lt[k][v] = l;
    }
    __syncthreads();
#pragma unroll 1
    for (int k8 = 0; k8 < kT; k8 += 8) {
      double x[8];  // eight rows of In in flight together (rows past n read as zero)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gk = k0 + k8 + u;
        x[u] = gk < n ? In[(long long)gk * m + ic] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2* row = reinterpret_cast<const double2*>(&lt[k8 + u][0]);
#pragma unroll
        for (int v2 = 0; v2 < kT / 2; ++v2) {
          const double2 l2 = row[v2];
          acc[2 * v2] += l2.x * x[u];
          acc[2 * v2 + 1] += l2.y * x[u];
        }
      }
    }
    __syncthreads();
  }
  if (i >= m) return;
#pragma unroll
  for (int v = 0; v < kT; ++v)
    if (nu0 + v < n) Out[(long long)(nu0 + v) * m + i] = acc[v];
}

// C = A B for n x n row-major upper triangular A and B (C upper): one thread per entry (a
// tiled version measured slower: its few blocks wait on dependent tile loads).
__global__ void k_trmm_small(const double* __restrict__ A, const double* __restrict__ B, int n,
                             double* __restrict__ C) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int r = (int)(e / n), c = (int)(e - (long long)r * n);
  double a = 0.0;
  for (int k = r; k <= c; ++k) a += A[(long long)r * n + k] * B[(long long)k * n + c];
  C[e] = a;
}

// Checks of the two Cholesky factors and the rank figures: q[0] = number of breakdowns,
// q[1] = max_i |R2_ii - 1|, q[2] = min / max |R_ii|; rd2 = (min, max) |R1_ii R2_ii| (the
// diagonal of R = R2 R1).
__global__ void k_cqr_check(const double* __restrict__ R1, const double* __restrict__ R2, int n,
                            const int* __restrict__ bad, double* __restrict__ q,
                            double* __restrict__ rd2) {
  __shared__ double smin[256], smax[256], sdev[256];
  double mn = INFINITY, mx = 0.0, dv = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double a = R1[(long long)k * n + k], b = R2[(long long)k * n + k];
    const double r = fabs(a * b);
    mn = fmin(mn, r);
    mx = fmax(mx, r);
    dv = fmax(dv, isfinite(b) ? fabs(b - 1.0) : INFINITY);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sdev[threadIdx.x] = dv;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      sdev[threadIdx.x] = fmax(sdev[threadIdx.x], sdev[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    q[0] = (double)(bad[0] + bad[1]);
    q[1] = sdev[0];
    q[2] = smax[0] > 0.0 ? smin[0] / smax[0] : 0.0;
    rd2[0] = smin[0];
    rd2[1] = smax[0];
  }
}

__global__ void k_cqr_flags_reset(int* bad) {
  if (threadIdx.x < 2) bad[threadIdx.x] = 0;
}

void syrk(const double* X, int m, int n, double* Gp, double* G, hipStream_t s) {
  const int nt = (n + kST - 1) / kST, pairs = nt * (nt + 1) / 2;
  const int nchunk = gram_chunks(m, n);
  const int rc = (m + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_syrk_part, dim3(pairs, nchunk), dim3(256), 0, s, X, m, n, rc, Gp);
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(k_syrk_reduce, dim3((unsigned)((nn + 3) / 4)), dim3(256), 0, s, Gp, nchunk,
                     n, G);
}

// R = chol(G) and X = R^-1: one launch per tile panel.
void chol_inv(const double* G, double* R, double* X, int n, int* bad, hipStream_t s) {
  const int nt = (n + kT - 1) / kT;
  for (int p = 0; p < nt; ++p)
    hipLaunchKernelGGL(k_chol_panel, dim3(nt + 1), dim3(256), 0, s, G, R, X, n, p, bad);
}

void tri_apply(bool trans, const double* Rm, int n, const double* In, int m, double* Out,
               hipStream_t s) {
  const dim3 grid((unsigned)((m + 255) / 256), (unsigned)((n + kT - 1) / kT));
  if (trans) hipLaunchKernelGGL(k_tri_apply<true>, grid, dim3(256), 0, s, Rm, n, In, m, Out);
  else hipLaunchKernelGGL(k_tri_apply<false>, grid, dim3(256), 0, s, Rm, n, In, m, Out);
}

}  // namespace

// Largest accepted max_i |R2_ii - 1| (pass 1's loss of orthogonality seen by pass 2), and the
// smallest accepted min / max |R_ii|: below it (the coupled Case 2 systems, kappa 1e8 - 1e10
// with columns of very different norms) CholeskyQR2's coefficients carried 50 - 100 times the
// Householder QR's error at the same residual in a NumPy emulation, while at the boundary
// matrices of one domain (kappa up to 5e4) the two agree.
constexpr double kCqrDev = 0.05;
constexpr double kCqrRdiag = 1e-5;

dpm_status cqr2_operator(double* A, int m, int n, double* P, const CqrScratch& w, double* rd2,
                         hipStream_t s, bool* used) {
  *used = false;
  if (n < 1 || m < n) { set_error("CholeskyQR2: need m >= n >= 1 (m = %d, n = %d)", m, n); return DPM_EINVAL; }
  hipLaunchKernelGGL(k_cqr_flags_reset, dim3(1), dim3(64), 0, s, w.bad);
  // pass 1: Q1^T = R1^-T A^T into P's buffer (A stays intact for the fallback)
  syrk(A, m, n, w.Gp, w.G, s);
  chol_inv(w.G, w.R1, w.Ri1, n, w.bad, s);
  tri_apply(true, w.Ri1, n, A, m, P, s);
  // pass 2: the Gram of Q1, its factor and inverse
  syrk(P, m, n, w.Gp, w.G, s);
  chol_inv(w.G, w.R2, w.Ri2, n, w.bad + 1, s);
  hipLaunchKernelGGL(k_cqr_check, dim3(1), dim3(256), 0, s, w.R1, w.R2, n, w.bad, w.q, rd2);
  DPM_TRY_HIP(hipGetLastError());
  double q[3] = {1.0, 0.0, 0.0};
  DPM_TRY_HIP(hipMemcpyAsync(q, w.q, sizeof(q), hipMemcpyDeviceToHost, s));
  DPM_TRY_HIP(hipStreamSynchronize(s));
  if (q[0] != 0.0 || !(q[1] <= kCqrDev) || !(q[2] >= kCqrRdiag)) return DPM_OK;  // Householder on A
  // Q^T = R2^-T Q1^T into A's buffer, R^-1 = R1^-1 R2^-1, P = R^-1 Q^T
  tri_apply(true, w.Ri2, n, P, m, A, s);
  hipLaunchKernelGGL(k_trmm_small, dim3((unsigned)(((long long)n * n + 255) / 256)), dim3(256), 0,
                     s, w.Ri1, w.Ri2, n, w.Ri);
  tri_apply(false, w.Ri, n, A, m, P, s);
  DPM_TRY_HIP(hipGetLastError());
  *used = true;
  return DPM_OK;
}

}  // namespace dpm
