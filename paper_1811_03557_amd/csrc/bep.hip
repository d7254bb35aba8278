// Boundary equations of the DPM on the device (paper Sec. 2 and Algorithm "Main Steps",
// Steps 2 and 5): right-hand sides of the difference potentials of the basis densities, the
// reduced-BEP matrix A[:, nu] = Tr_gamma_in (I - P_gamma) phi_nu (eq BEP_recast), its FP64
// Householder QR, and the least-squares solve C = R^-1 Q^T g.
#include <cmath>
#include <vector>

#include "bep.h"

namespace dpm {

dpm_status gamma_points_impl(const dpm_grid& g, const uint8_t* m_plus, int32_t* n_gamma,
                             int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, hipStream_t s);

namespace {

constexpr int kB = 256;

__global__ void k_fill_zero(double* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// gpos[i] = position of node i in the gamma list, or -1.
__global__ void k_gpos(const int32_t* __restrict__ idx, int ng, int32_t* __restrict__ gpos,
                       long long vsz, int phase) {
  if (phase == 0) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vsz;
         i += (long long)gridDim.x * blockDim.x)
      gpos[i] = -1;
  } else {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ng) gpos[idx[k]] = k;
  }
}

// out[c][q] = (sigma - Lap_h)[v_c] at the M- nodes q where it can be nonzero, v_c the density
// dens[c0 + c] on gamma extended by zero (zero Dirichlet data outside the cube), c < ncol.
// Those nodes are gamma_ex and the M- neighbours of gamma_ex (an M- neighbour of a gamma_in node
// is in gamma_ex): thread (e, k) takes gamma node e, if it is in gamma_ex, and its k-th node of
// {itself, 6 neighbours}, finds the gamma positions of that node's stencil once and then
// writes every column; a node reached from two gamma_ex nodes gets the same value twice.  The
// set of nodes written depends only on the geometry.  Other entries of out are left as they
// are (the caller has them at zero on M-).
__global__ void k_minus_rhs(const double* __restrict__ dens, int c0, int ncol, int ng,
                            const int32_t* __restrict__ idx, const uint8_t* __restrict__ is_in,
                            const int32_t* __restrict__ gpos, const uint8_t* __restrict__ mp,
                            int n, double sigma, double inv_h2, double* __restrict__ out,
                            long long vsz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = t / 7, k = t - 7 * (t / 7);
  if (e >= ng || is_in[e]) return;
  const unsigned p = (unsigned)idx[e], un = (unsigned)n;
  int x = (int)(p % un), y = (int)((p / un) % un), z = (int)(p / (un * un));
  // k: 0 self, 1/2 x-+, 3/4 y-+, 5/6 z-+
  if (k == 1) --x; else if (k == 2) ++x; else if (k == 3) --y; else if (k == 4) ++y;
  else if (k == 5) --z; else if (k == 6) ++z;
  if (x < 0 || x >= n || y < 0 || y >= n || z < 0 || z >= n) return;
  const long long q = ((long long)z * n + y) * n + x;
  if (mp[q]) return;
  // gamma positions of the node and its in-cube neighbours (-1: not on gamma or outside)
  const long long nn = (long long)n * n;
  const int g0 = gpos[q];
  const int gx0 = x > 0 ? gpos[q - 1] : -1, gx1 = x < n - 1 ? gpos[q + 1] : -1;
  const int gy0 = y > 0 ? gpos[q - n] : -1, gy1 = y < n - 1 ? gpos[q + n] : -1;
  const int gz0 = z > 0 ? gpos[q - nn] : -1, gz1 = z < n - 1 ? gpos[q + nn] : -1;
  const double diag = sigma + 6.0 * inv_h2;
  for (int c = 0; c < ncol; ++c) {
    const double* dr = dens + (long long)(c0 + c) * ng;
    auto at = [&](int gi) { return gi >= 0 ? dr[gi] : 0.0; };
    const double nb = at(gx0) + at(gx1) + at(gy0) + at(gy1) + at(gz0) + at(gz1);
    out[(long long)c * vsz + q] = diag * at(g0) - inv_h2 * nb;
  }
}

// A[i + (c0+c)*n_in] = dens[(c0+c)][pos_in[i]] - u[c][idx_in[i]]
__global__ void k_trace_columns(const double* __restrict__ dens, const double* __restrict__ u,
                                const int32_t* __restrict__ idx_in,
                                const int32_t* __restrict__ pos_in, int n_in, int ng, int c0,
                                int ncol, long long vsz, double* __restrict__ A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n_in || c >= ncol) return;
  A[(long long)(c0 + c) * n_in + i] =
      dens[(long long)(c0 + c) * ng + pos_in[i]] - u[(long long)c * vsz + idx_in[i]];
}

__device__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += sh[k];  // fixed order: deterministic
  return t;
}

// Sums of two values over the block, in a fixed order (deterministic).
__device__ void block_sum2(double& a, double& b, double* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { sh[2 * w] = a; sh[2 * w + 1] = b; }
  __syncthreads();
  double s = 0.0, t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) { s += sh[2 * k]; t += sh[2 * k + 1]; }
  a = s;
  b = t;
}

// Threads of a Householder step; each holds R rows of a column in registers (rows p + 1 + t +
// u * kQT for the pivot p), and rows beyond R * kQT are streamed in a second loop.
constexpr int kQT = 1024;

// Householder reflector (LAPACK dlarfg convention) of a column x at pivot p, from alpha = x_p
// and sigma2 = ||x[p+1:]||^2: beta = -sign(alpha) sqrt(alpha^2 + sigma2), v_p = 1,
// v_i = x_i / (alpha - beta) (i > p), tau = (beta - alpha) / beta; sigma2 = 0 means H = I
// (tau = 0, v not stored).
struct Refl {
  double beta, scal, tau;
};
__device__ __forceinline__ Refl make_refl(double alpha, double sigma2) {
  const double nrm = sqrt(alpha * alpha + sigma2);
  Refl r;
  r.beta = alpha >= 0.0 ? -nrm : nrm;
  r.scal = 1.0 / (alpha - r.beta);
  r.tau = (r.beta - alpha) / r.beta;
  return r;
}

// One step j of the Householder QR in place.  Blocks 1.. apply H_j, formed from the raw column
// j, to the trailing columns k = j + blockIdx.x: one pass loads x = A[j+1:, j] and a =
// A[j+1:, k] and reduces ||x||^2 and x^T a together, so that v^T a = a_j + scal x^T a.
// Block 0 stores the reflector of the previous step (column j - 1, which no other block of
// this launch reads): A[j-1, j-1] = beta (= R), A[j:, j-1] = v, tau[j-1].  Launched for
// j = 0..n (the last launch only stores step n - 1).  Every block forms the reflector from the
// same values in the same order, so the stored v is the one that was applied.
template <int R>
__global__ __launch_bounds__(kQT) void k_house_step(double* __restrict__ A, int m, int ncols,
                                                    int j, double* __restrict__ tau) {
  __shared__ double sh[2 * (kQT / 64)];
  const int t = threadIdx.x;
  const bool store = blockIdx.x == 0;
  const int p = store ? j - 1 : j;  // pivot of the reflector this block forms
  const int k = j + blockIdx.x;
  if (store ? j == 0 : (j >= ncols || k >= ncols)) return;
  double* c = A + (long long)p * m;
  double* a = A + (long long)k * m;  // block 0: unused
  const int r0 = p + 1;
  double x[R], y[R];
  double ss = 0.0, xa = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = r0 + t + u * kQT;
    x[u] = i < m ? c[i] : 0.0;
    y[u] = (!store && i < m) ? a[i] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < R; ++u) { ss += x[u] * x[u]; xa += x[u] * y[u]; }
  for (int i = r0 + R * kQT + t; i < m; i += kQT) {  // rows beyond the register tile
    const double xi = c[i];
    ss += xi * xi;
    if (!store) xa += xi * a[i];
  }
  block_sum2(ss, xa, sh);
  const double alpha = c[p];
  if (ss == 0.0) {  // H = I
    if (store && t == 0) tau[p] = 0.0;
    return;
  }
  const Refl h = make_refl(alpha, ss);
  if (store) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = r0 + t + u * kQT;
      if (i < m) c[i] = x[u] * h.scal;
    }
    for (int i = r0 + R * kQT + t; i < m; i += kQT) c[i] *= h.scal;
    if (t == 0) {
      c[p] = h.beta;
      tau[p] = h.tau;
    }
    return;
  }
  const double aj = a[j];
  const double w = h.tau * (aj + h.scal * xa);
  if (t == 0) a[j] = aj - w;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = r0 + t + u * kQT;
    if (i < m) a[i] = y[u] - w * (x[u] * h.scal);
  }
  for (int i = r0 + R * kQT + t; i < m; i += kQT) a[i] -= w * (c[i] * h.scal);
}

// Rows per thread of the register tile for the rows below pivot j.
int qr_rows_per_thread(int m, int j) {
  const int rows = m - j;
  for (int r : {1, 2, 4, 8, 12, 16})
    if (r * kQT >= rows) return r;
  return 20;  // the largest tile without spills at kQT threads
}

void launch_house_step(double* A, int m, int ncols, int j, double* tau, hipStream_t s) {
  const dim3 grid(j < ncols ? ncols - j : 1), block(kQT);
  switch (qr_rows_per_thread(m, j > 0 ? j - 1 : 0)) {
    case 1: hipLaunchKernelGGL(k_house_step<1>, grid, block, 0, s, A, m, ncols, j, tau); break;
    case 2: hipLaunchKernelGGL(k_house_step<2>, grid, block, 0, s, A, m, ncols, j, tau); break;
    case 4: hipLaunchKernelGGL(k_house_step<4>, grid, block, 0, s, A, m, ncols, j, tau); break;
    case 8: hipLaunchKernelGGL(k_house_step<8>, grid, block, 0, s, A, m, ncols, j, tau); break;
    case 12: hipLaunchKernelGGL(k_house_step<12>, grid, block, 0, s, A, m, ncols, j, tau); break;
    case 16: hipLaunchKernelGGL(k_house_step<16>, grid, block, 0, s, A, m, ncols, j, tau); break;
    default: hipLaunchKernelGGL(k_house_step<20>, grid, block, 0, s, A, m, ncols, j, tau); break;
  }
}

// Compact WY form of the reflectors (Schreiber-Van Loan): Q = H_0 ... H_{n-1} = I - V T V^T,
// V (m x n) unit lower trapezoidal (the Householder vectors below R in A, with the implicit
// unit diagonal), T (n x n) upper triangular.
__device__ __forceinline__ double vval(const double* __restrict__ A, int m, int i, int k) {
  return i == k ? 1.0 : (i > k ? A[(long long)k * m + i] : 0.0);
}

// G = V^T V (n x n, row-major), upper triangle of 32 x 32 tiles (tile row <= tile column), the
// rows of V split into chunks of rc rows over blockIdx.y: block (tile, chunk) writes its
// partial sum to Gp[chunk], k_gram_reduce adds the chunks in order (deterministic).  Rows of a
// chunk are staged through LDS 32 at a time; each thread owns a 2 x 2 block of the tile.
constexpr int kGT = 32;
__global__ __launch_bounds__(256) void k_gram_part(const double* __restrict__ A, int m, int n,
                                                   int rc, double* __restrict__ Gp) {
  __shared__ double va[kGT][kGT + 1], vb[kGT][kGT + 1];  // [row][column]
  const int nt = (n + kGT - 1) / kGT;
  // tile index -> (ta, tb), ta <= tb, row-major over the upper triangle
  int tile = blockIdx.x, ta = 0;
  while (tile >= nt - ta) { tile -= nt - ta; ++ta; }
  const int tb = ta + tile;
  const int a0 = ta * kGT, b0 = tb * kGT;
  const int i_lo = blockIdx.y * rc, i_hi = min(m, i_lo + rc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // outputs (a0+2tx+{0,1}, b0+2ty+{0,1})
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  const int start = max(i_lo, b0);  // V[i][k] = 0 for i < k, and b0 >= a0
  const int lr = threadIdx.x & 31, lc = threadIdx.x >> 5;  // loader: row lr, columns lc + 8q
  for (int i0 = start; i0 < i_hi; i0 += kGT) {
    const int i = i0 + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ca = a0 + lc + 8 * q, cb = b0 + lc + 8 * q;
      va[lr][lc + 8 * q] = (i < i_hi && ca < n) ? vval(A, m, i, ca) : 0.0;
      vb[lr][lc + 8 * q] = (i < i_hi && cb < n) ? vval(A, m, i, cb) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < kGT; ++r) {
      const double x0 = va[r][2 * tx], x1 = va[r][2 * tx + 1];
      const double y0 = vb[r][2 * ty], y1 = vb[r][2 * ty + 1];
      acc[0][0] += x0 * y0;
      acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0;
      acc[1][1] += x1 * y1;
    }
    __syncthreads();
  }
  double* g = Gp + (long long)blockIdx.y * n * n;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int ra = a0 + 2 * tx + u, cb = b0 + 2 * ty + v;
      if (ra < n && cb < n) g[(long long)ra * n + cb] = acc[u][v];
    }
}

// G[a][b] = sum over chunks of Gp[chunk][a][b], for a <= b (the part k_tinv reads): one
// wavefront per entry, lane l adding chunks l, l + 64, ..., then a fixed butterfly across the
// lanes (the same order every run).
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ Gp, int nchunk,
                                                     int n, double* __restrict__ G) {
  const long long e = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= (long long)n * n) return;  // uniform across the wavefront
  const int ra = (int)(e / n), cb = (int)(e - (long long)ra * n);
  // entries with a > b are not written by k_gram_part (and not read)
  if (ra > cb) {
    if (lane == 0) G[e] = 0.0;
    return;
  }
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += Gp[(long long)c * n * n + e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) G[e] = s;
}

// T (row-major, upper triangular).  With tau_j = 2 / (v_j^T v_j) (every reflector here, or
// tau_j = 0), T^-1 is the upper triangle of G with 1/tau_j on the diagonal, so column c of T
// solves that triangle against e_c: x_j = tau_j (delta_jc - sum_{j < k <= c} G[j][k] x_k),
// which also gives a zero column for tau_j = 0.  One block per column.
__global__ void k_tinv(const double* __restrict__ G, const double* __restrict__ tau, int n,
                       double* __restrict__ T) {
  __shared__ double sh[16];
  __shared__ double x[1024];
  const int c = blockIdx.x;
  for (int k = threadIdx.x; k < n; k += blockDim.x) x[k] = 0.0;
  __syncthreads();
  for (int j = c; j >= 0; --j) {
    double d = 0.0;
    for (int k = j + 1 + threadIdx.x; k <= c; k += blockDim.x) d += G[(long long)j * n + k] * x[k];
    const double s = block_sum(d, sh);
    if (threadIdx.x == 0) x[j] = tau[j] * ((j == c ? 1.0 : 0.0) - s);
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) T[(long long)k * n + c] = x[k];
}

// W = V1 T^T with V1 = V[0:n, 0:n] (unit lower triangular): W[a][b] = sum_k V1[a][k] T[b][k],
// nonzero terms for b <= k <= a.  One thread per entry.
__global__ void k_v1tt(const double* __restrict__ A, int m, int n, const double* __restrict__ T,
                       double* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int a = e / n, bcol = e - a * n;
  double d = 0.0;
  for (int k = bcol; k <= a; ++k) d += vval(A, m, a, k) * T[(long long)bcol * n + k];
  W[e] = d;
}

// K = Rinv W (Rinv upper triangular: terms a >= nu).  One thread per entry.
__global__ void k_kmat(const double* __restrict__ Rinv, const double* __restrict__ W, int n,
                       double* __restrict__ K) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int nu = e / n, bcol = e - nu * n;
  double d = 0.0;
  for (int a = nu; a < n; ++a) d += Rinv[(long long)nu * n + a] * W[(long long)a * n + bcol];
  K[e] = d;
}

// Rinv = R^-1 (n x n, row-major, upper triangular) with R the upper triangle of A: one block
// per column c, back substitution R x = e_c with the dot products reduced across the block.
__global__ void k_rinv(const double* __restrict__ A, int m, int n, double* __restrict__ Rinv) {
  __shared__ double sh[16];
  __shared__ double x[1024];
  const int c = blockIdx.x;
  for (int k = threadIdx.x; k < n; k += blockDim.x) x[k] = 0.0;
  __syncthreads();
  for (int nu = c; nu >= 0; --nu) {
    double d = 0.0;
    for (int k = nu + 1 + threadIdx.x; k <= c; k += blockDim.x) d += A[(long long)k * m + nu] * x[k];
    const double s = block_sum(d, sh);
    if (threadIdx.x == 0) x[nu] = ((nu == c ? 1.0 : 0.0) - s) / A[(long long)nu * m + nu];
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) Rinv[(long long)k * n + c] = x[k];
}

// P = R^-1 Q1^T = [Rinv 0] - K V^T (Q1 = [I; 0] - V T V1^T): P[nu][i] = Rinv[nu][i] (i < n)
// - sum_{k <= min(i, n-1)} K[nu][k] V[i][k], for a tile of PT rows nu (K rows in LDS) and one
// row i of V per thread (V[i][k] = A[k m + i], coalesced across threads).
constexpr int PT = 8;
__global__ void k_form_p(const double* __restrict__ Rinv, const double* __restrict__ K,
                         const double* __restrict__ A, int m, int n, double* __restrict__ P) {
  extern __shared__ double kt[];  // PT x n
  const int nu0 = blockIdx.y * PT;
  for (int t = threadIdx.x; t < PT * n; t += blockDim.x) {
    const int r = t / n, k = t - r * n;
    kt[t] = nu0 + r < n ? K[(long long)(nu0 + r) * n + k] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) acc[t] = 0.0;
  const int kend = i < n - 1 ? i : n - 1;
  for (int k = 0; k <= kend; ++k) {
    const double v = vval(A, m, i, k);
#pragma unroll
    for (int t = 0; t < PT; ++t) acc[t] += kt[t * n + k] * v;
  }
#pragma unroll
  for (int t = 0; t < PT; ++t)
    if (nu0 + t < n)
      P[(long long)(nu0 + t) * m + i] = (i < n ? Rinv[(long long)(nu0 + t) * n + i] : 0.0) - acc[t];
}

// C[r][nu] = sum_i P[nu][i] g_r[i]: the least-squares coefficients of right-hand side r, with
// g_r[i] = g[r m + i], or, gathering, g_r[i] = vol[r vsz + idx[i]] (the trace of solution r on
// gamma_in read straight from its volume).  One block of kLT threads per (nu, r); each thread
// loads kLU rows at a time, all in flight together, then one fixed-order block reduction.
constexpr int kLT = 1024, kLU = 16;
template <bool GATHER>
__global__ __launch_bounds__(kLT) void k_lsq_apply(const double* __restrict__ P, int m, int n,
                                                   const double* __restrict__ g, long long vsz,
                                                   const int32_t* __restrict__ idx,
                                                   double* __restrict__ C) {
  __shared__ double sh[kLT / 64];
  const int nu = blockIdx.x, r = blockIdx.y;
  const double* pr = P + (long long)nu * m;
  double d = 0.0;
  for (int b0 = 0; b0 < m; b0 += kLU * kLT) {
    double pv[kLU], gv[kLU];
#pragma unroll
    for (int u = 0; u < kLU; ++u) {
      const int i = b0 + threadIdx.x + u * kLT;
      pv[u] = i < m ? pr[i] : 0.0;
      if (GATHER)
        gv[u] = i < m ? g[(long long)r * vsz + idx[i]] : 0.0;
      else
        gv[u] = i < m ? g[(long long)r * m + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLU; ++u) d += pv[u] * gv[u];
  }
  const double t = block_sum(d, sh);
  if (threadIdx.x == 0) C[(long long)r * n + nu] = t;
}

// out2 = (min |R_ii|, max |R_ii|) over the diagonal of the factored A (one block); a NaN on the
// diagonal makes both NaN, so the rank test fails.
__global__ __launch_bounds__(256) void k_rdiag_minmax(const double* __restrict__ A, int m, int n,
                                                      double* __restrict__ out2) {
  __shared__ double smn[4], smx[4];
  __shared__ int snan[4];
  double mn = INFINITY, mx = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = fabs(A[(long long)i * m + i]);
    bad |= !(v == v);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
    bad |= __shfl_xor(bad, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { smn[w] = mn; smx[w] = mx; snan[w] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) { mn = fmin(mn, smn[k]); mx = fmax(mx, smx[k]); bad |= snan[k]; }
    out2[0] = bad ? NAN : mn;
    out2[1] = bad ? NAN : mx;
  }
}

// positions of the gamma_in entries inside the gamma list, and their linear indices
__global__ void k_in_lists(const int32_t* __restrict__ idx, const uint8_t* __restrict__ is_in,
                           const int32_t* __restrict__ rank_in, int ng,
                           int32_t* __restrict__ idx_in, int32_t* __restrict__ pos_in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ng && is_in[i]) {
    const int r = rank_in[i];
    idx_in[r] = idx[i];
    pos_in[r] = i;
  }
}

// N+ = M+ plus gamma_ex
__global__ void k_nplus(const uint8_t* __restrict__ mp, const int32_t* __restrict__ idx, int ng,
                        uint8_t* __restrict__ np, long long vsz, int phase) {
  if (phase == 0) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vsz;
         i += (long long)gridDim.x * blockDim.x)
      np[i] = mp[i];
  } else {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ng) np[idx[i]] = 1;
  }
}

unsigned grid1(long long n, int b = kB) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void fill_zero(double* p, long long n, hipStream_t s) {
  long long blocks = (n + kB - 1) / kB;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kB), 0, s, p, n);
}

void minus_rhs(const dpm_bep* b, const double* dens, int c0, int ncol, double* out,
               hipStream_t s) {
  const dpm_grid& g = b->grid;
  const long long vsz = (long long)g.n * g.n * g.n;
  hipLaunchKernelGGL(k_minus_rhs, dim3(grid1(7LL * b->n_gamma)), dim3(kB), 0, s, dens, c0, ncol,
                     b->n_gamma, b->idx, b->is_in, b->gpos, b->m_plus, g.n, g.sigma,
                     1.0 / (g.h * g.h), out, vsz);
}

void qr_solve(const dpm_bep* bep, int nvec, const double* g, double* C, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_apply<false>, dim3(bep->n_basis, nvec), dim3(kLT), 0, s, bep->P,
                     bep->n_in, bep->n_basis, g, 0LL, nullptr, C);
}

void lsq_apply(const double* P, int m, int n, int nvec, const double* g, double* C,
               hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_apply<false>, dim3(n, nvec), dim3(kLT), 0, s, P, m, n, g, 0LL,
                     nullptr, C);
}

void qr_solve_traces(const dpm_bep* bep, int nvec, const double* vol, long long vsz, double* C,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_apply<true>, dim3(bep->n_basis, nvec), dim3(kLT), 0, s, bep->P,
                     bep->n_in, bep->n_basis, vol, vsz, bep->idx_in, C);
}

// Row chunks of the Gram product: about 2,048 blocks over the upper-triangle tiles, chunks of
// 32 to 1,024 rows.
int gram_chunks(int m, int n) {
  const int nt = (n + kGT - 1) / kGT, tiles = nt * (nt + 1) / 2;
  int rc = (int)(((long long)m * tiles + 2047) / 2048);
  rc = rc < 32 ? 32 : (rc > 1024 ? 1024 : rc);
  return (m + rc - 1) / rc;
}

namespace {

// Columns per batched solve of a build: 16, fewer where the right-hand sides and solutions of
// 16 columns (2 x 16 FP64 volumes) would pass 2 GiB; opts->rhs_chunk overrides.
int build_cols(const dpm_grid& g, const dpm_opts& o, int n_basis) {
  const double per = 16.0 * (double)g.n * g.n * g.n;
  int c = o.rhs_chunk > 0 ? o.rhs_chunk : (int)std::fmin(16.0, std::floor(2147483648.0 / per));
  if (c > n_basis) c = n_basis;
  return c < 1 ? 1 : c;
}

struct ColLayout {
  int chunk;
  size_t rhs, u, ws, wsb, total;
};
ColLayout col_layout(const dpm_grid& g, const dpm_opts& o, int n_basis) {
  ColLayout L{};
  L.chunk = build_cols(g, o, n_basis);
  const size_t vb = sizeof(double) * (size_t)g.n * g.n * g.n * (size_t)L.chunk;
  dpm_opts so = o;
  so.rhs_chunk = 0;
  size_t wsb = 0;
  (void)workspace_size_impl(g, L.chunk, so, &wsb);
  size_t at = 0;
  L.rhs = at; at = align_up(at + vb, 256);
  L.u = at; at = align_up(at + vb, 256);
  L.ws = at; L.wsb = wsb; at = align_up(at + wsb, 256);
  L.total = at;
  return L;
}

struct FacLayout {
  size_t rd, G, T, W, K, Rinv, Gp, Ws, Vs, inv, flg, Ri, cq, total;
};
FacLayout fac_layout(int m, int n) {
  const size_t nn = sizeof(double) * (size_t)n * n;
  const SvdShape sh = svd_shape(n);
  const size_t npp = sizeof(double) * (size_t)sh.np * sh.np;
  FacLayout L{};
  size_t at = 0;
  L.rd = at; at = align_up(at + 4 * sizeof(double), 256);
  L.G = at; at = align_up(at + nn, 256);
  L.T = at; at = align_up(at + nn, 256);
  L.W = at; at = align_up(at + nn, 256);
  L.K = at; at = align_up(at + nn, 256);
  L.Rinv = at; at = align_up(at + nn, 256);
  L.Gp = at; at = align_up(at + nn * (size_t)gram_chunks(m, n), 256);
  // truncated least squares (rcond > 0): the Jacobi SVD's W, V, inverse squares and flags
  L.Ws = at; at = align_up(at + npp, 256);
  L.Vs = at; at = align_up(at + npp, 256);
  L.inv = at; at = align_up(at + sizeof(double) * (size_t)n, 256);
  L.flg = at; at = align_up(at + 3 * sizeof(unsigned long long), 256);
  // CholeskyQR2: R^-1, then two check values and two breakdown counters
  L.Ri = at; at = align_up(at + nn, 256);
  L.cq = at; at = align_up(at + 3 * sizeof(double) + 2 * sizeof(int), 256);
  L.total = at;
  return L;
}

}  // namespace

size_t columns_scratch_bytes(const dpm_bep* b) {
  return col_layout(b->grid, b->opts, b->n_basis).total;
}
size_t factor_scratch_bytes(int m, int n) { return fac_layout(m, n).total; }
size_t rebuild_scratch_bytes(const dpm_bep* b) {
  const size_t c = columns_scratch_bytes(b), f = factor_scratch_bytes(b->n_in, b->n_basis);
  return c > f ? c : f;  // the factorisation starts after the column solves: shared scratch
}

dpm_status rank_check(double mn, double mx) {
  if (!(mn > 1e-12 * mx)) {
    set_error("boundary matrix is rank deficient: min |R_ii| = %g, max |R_ii| = %g", mn, mx);
    return DPM_ERANK;
  }
  return DPM_OK;
}

// Columns of the reduced-BEP matrix at the handle's sigma (M- operator on the densities, batched
// AP solves, traces on gamma_in) into b->A, with the right-hand sides, solutions and solve
// workspace taken from `scratch` (columns_scratch_bytes).  Enqueue only: no allocation and no
// synchronisation.
dpm_status bep_columns(dpm_bep* b, hipStream_t s, void* scratch, size_t bytes) {
  const dpm_grid& g = b->grid;
  const int n_basis = b->n_basis, nin = b->n_in, ng = b->n_gamma;
  const long long vsz = (long long)g.n * g.n * g.n;
  const ColLayout L = col_layout(g, b->opts, n_basis);
  if (scratch == nullptr || bytes < L.total) {
    set_error("boundary-matrix columns: scratch too small: %zu bytes given, %zu needed", bytes,
              L.total);
    return DPM_EINVAL;
  }
  char* base = static_cast<char*>(scratch);
  double* rhs = reinterpret_cast<double*>(base + L.rhs);
  double* u = reinterpret_cast<double*>(base + L.u);
  dpm_opts so = b->opts;
  so.workspace = base + L.ws;
  so.workspace_bytes = L.wsb;
  so.rhs_chunk = 0;
  const int chunk = L.chunk;
  for (int c0 = 0; c0 < n_basis; c0 += chunk) {
    const int nc = (n_basis - c0) < chunk ? (n_basis - c0) : chunk;
    // zeros once: every chunk writes the same nodes (the set depends on the geometry only) and
    // the solves leave their right-hand sides unchanged
    if (c0 == 0) fill_zero(rhs, vsz * nc, s);
    minus_rhs(b, b->basis, c0, nc, rhs, s);
    DPM_TRY(aux_solve_impl(g, nc, rhs, u, so, s, nullptr));
    hipLaunchKernelGGL(k_trace_columns, dim3(grid1(nin), nc), dim3(kB), 0, s, b->basis, u,
                       b->idx_in, b->pos_in, nin, ng, c0, nc, vsz, b->A);
    DPM_TRY_HIP(hipGetLastError());
  }
  return DPM_OK;
}

// Householder QR of A (m x n, column-major, overwritten by the reflectors below R), the least-
// squares operator P = R^-1 Q1^T (n x m, row nu contiguous) and (min, max) |R_ii| into the device
// pair rd2, with temporaries from `scratch` (factor_scratch_bytes).  Enqueue only: the caller
// reads rd2 back for the rank test.
dpm_status lsq_factor(double* A, int m, int n_basis, double* tau, double* P, hipStream_t s,
                      void* scratch, size_t bytes, double* rd2, double rcond, int* method) {
  const int nin = m;
  const FacLayout L = fac_layout(m, n_basis);
  if (scratch == nullptr || bytes < L.total) {
    set_error("least-squares factorisation: scratch too small: %zu bytes given, %zu needed", bytes,
              L.total);
    return DPM_EINVAL;
  }
  char* base = static_cast<char*>(scratch);
  if (rcond <= 0.0) {
    // CholeskyQR2 (BLAS-3 shaped); the Householder QR below when it reports a breakdown or a
    // matrix too ill-conditioned for it (A is then untouched)
    CqrScratch w;
    w.Gp = reinterpret_cast<double*>(base + L.Gp);
    w.G = reinterpret_cast<double*>(base + L.G);
    w.R1 = reinterpret_cast<double*>(base + L.T);
    w.R2 = reinterpret_cast<double*>(base + L.W);
    w.Ri1 = reinterpret_cast<double*>(base + L.K);
    w.Ri2 = reinterpret_cast<double*>(base + L.Rinv);
    w.Ri = reinterpret_cast<double*>(base + L.Ri);
    w.q = reinterpret_cast<double*>(base + L.cq);
    w.bad = reinterpret_cast<int*>(base + L.cq + 3 * sizeof(double));
    bool used = false;
    DPM_TRY(cqr2_operator(A, nin, n_basis, P, w, rd2, s, &used));
    if (used) {
      if (method) *method = DPM_LSQ_CHOLESKY_QR2;
      return DPM_OK;
    }
  }
  if (method) *method = rcond > 0.0 ? DPM_LSQ_HOUSEHOLDER_TRUNCATED : DPM_LSQ_HOUSEHOLDER;
  // one launch per step (the step-j reflector is applied by the trailing-column blocks and
  // stored by block 0 of the next launch)
  for (int j = 0; j <= n_basis; ++j) launch_house_step(A, nin, n_basis, j, tau, s);
  hipLaunchKernelGGL(k_rdiag_minmax, dim3(1), dim3(256), 0, s, A, nin, n_basis, rd2);
  // least-squares operator P = R^-1 Q1^T, so that every later solve is one product C = P g
  const size_t nn = (size_t)n_basis * n_basis;
  double* G = reinterpret_cast<double*>(base + L.G);
  double* T = reinterpret_cast<double*>(base + L.T);
  double* W = reinterpret_cast<double*>(base + L.W);
  double* K = reinterpret_cast<double*>(base + L.K);
  double* Rinv = reinterpret_cast<double*>(base + L.Rinv);
  double* Gp = reinterpret_cast<double*>(base + L.Gp);
  const int nt = (n_basis + kGT - 1) / kGT, nchunk = gram_chunks(nin, n_basis);
  const int rc = (nin + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_gram_part, dim3(nt * (nt + 1) / 2, nchunk), dim3(256), 0, s, A, nin,
                     n_basis, rc, Gp);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((nn + 3) / 4)), dim3(256), 0, s, Gp,
                     nchunk, n_basis, G);
  hipLaunchKernelGGL(k_tinv, dim3(n_basis), dim3(256), 0, s, G, tau, n_basis, T);
  hipLaunchKernelGGL(k_v1tt, dim3(grid1((long long)nn)), dim3(kB), 0, s, A, nin, n_basis, T, W);
  if (rcond > 0.0) {
    // truncated pseudo-inverse of R in place of R^-1 (a general, not triangular, matrix)
    DPM_TRY(pinv_of_r(A, nin, n_basis, rcond, Rinv, reinterpret_cast<double*>(base + L.Ws),
                      reinterpret_cast<double*>(base + L.Vs), reinterpret_cast<double*>(base + L.inv),
                      reinterpret_cast<unsigned long long*>(base + L.flg), rd2, s));
    kmat_full(Rinv, W, n_basis, K, s);
  } else {
    hipLaunchKernelGGL(k_rinv, dim3(n_basis), dim3(256), 0, s, A, nin, n_basis, Rinv);
    hipLaunchKernelGGL(k_kmat, dim3(grid1((long long)nn)), dim3(kB), 0, s, Rinv, W, n_basis, K);
  }
  hipLaunchKernelGGL(k_form_p, dim3(grid1(nin), (n_basis + PT - 1) / PT), dim3(kB),
                     sizeof(double) * PT * n_basis, s, Rinv, K, A, nin, n_basis, P);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

// Columns, QR and least-squares operator of the handle's matrix (enqueue only), (min, max)
// |R_ii| into rd2.
dpm_status factor_bep_enqueue(dpm_bep* b, hipStream_t s, double* A_out, void* scratch,
                              size_t bytes, double* rd2) {
  DPM_TRY(bep_columns(b, s, scratch, bytes));
  if (A_out && hipMemcpyAsync(A_out, b->A, sizeof(double) * (size_t)b->n_basis * b->n_in,
                              hipMemcpyDeviceToDevice, s) != hipSuccess) {
    set_error("dpm_build_boundary_matrix: copy of A failed");
    return DPM_EHIP;
  }
  return lsq_factor(b->A, b->n_in, b->n_basis, b->tau, b->P, s, scratch, bytes, rd2, 0.0,
                    &b->lsq_method);
}

// The same, then one synchronisation for the rank test (rd2 read back from the end of scratch).
dpm_status factor_bep(dpm_bep* b, hipStream_t s, double* A_out, void* scratch, size_t bytes) {
  double* rd2 = reinterpret_cast<double*>(static_cast<char*>(scratch) + fac_layout(b->n_in, b->n_basis).rd);
  DPM_TRY(factor_bep_enqueue(b, s, A_out, scratch, bytes, rd2));
  double h2[2] = {0.0, 0.0};
  DPM_TRY_HIP(hipMemcpyAsync(h2, rd2, sizeof(h2), hipMemcpyDeviceToHost, s));
  DPM_TRY_HIP(hipStreamSynchronize(s));
  b->rdiag_min = h2[0];
  b->rdiag_max = h2[1];
  return rank_check(h2[0], h2[1]);
}

dpm_status build_bep_impl(const dpm_grid& g, const uint8_t* m_plus, int n_basis,
                          const double* basis, const dpm_opts& o, hipStream_t s, dpm_bep** out,
                          double* A_out, bool factor) {
  int32_t ng = 0, nin = 0;
  DPM_TRY(gamma_points_impl(g, m_plus, &ng, &nin, nullptr, nullptr, s));
  if (n_basis > nin) {
    set_error("n_basis = %d exceeds |gamma_in| = %d", n_basis, nin);
    return DPM_ERANK;
  }
  const long long vsz = (long long)g.n * g.n * g.n;
  dpm_bep* b = new dpm_bep();
  b->grid = g;
  b->n_gamma = ng;
  b->n_in = nin;
  b->n_basis = n_basis;
  b->opts = o;
  b->opts.workspace = nullptr;
  b->opts.workspace_bytes = 0;
  auto fail = [&](dpm_status st) {
    destroy_bep(b);
    return st;
  };
  auto al = [&](void** p, size_t bytes) { return hipMalloc(p, bytes > 0 ? bytes : 1) == hipSuccess; };
  if (!al((void**)&b->m_plus, vsz) || !al((void**)&b->n_plus, vsz) ||
      !al((void**)&b->idx, sizeof(int32_t) * ng) || !al((void**)&b->is_in, ng) ||
      !al((void**)&b->idx_in, sizeof(int32_t) * nin) ||
      !al((void**)&b->pos_in, sizeof(int32_t) * nin) ||
      !al((void**)&b->in_zoff, sizeof(int32_t) * (g.n + 1)) ||
      !al((void**)&b->basis, sizeof(double) * (size_t)n_basis * ng) ||
      !al((void**)&b->A, sizeof(double) * (size_t)n_basis * nin) ||
      !al((void**)&b->tau, sizeof(double) * n_basis) ||
      !al((void**)&b->P, sizeof(double) * (size_t)n_basis * nin) ||
      !al((void**)&b->gpos, sizeof(int32_t) * vsz)) {
    set_error("dpm_build_boundary_matrix: device allocation failed");
    return fail(DPM_ENOMEM);
  }
  if (hipMemcpyAsync(b->m_plus, m_plus, vsz, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b->basis, basis, sizeof(double) * (size_t)n_basis * ng,
                     hipMemcpyDeviceToDevice, s) != hipSuccess) {
    set_error("dpm_build_boundary_matrix: copy failed");
    return fail(DPM_EHIP);
  }
  {
    dpm_status st = gamma_points_impl(g, b->m_plus, &ng, &nin, b->idx, b->is_in, s);
    if (st != DPM_OK) return fail(st);
  }
  // gamma_in lists: rank of each gamma_in entry via a host scan of the flags
  {
    std::vector<uint8_t> fl(ng);
    std::vector<int32_t> rk(ng, 0);
    if (hipMemcpy(fl.data(), b->is_in, ng, hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("dpm_build_boundary_matrix: copy failed");
      return fail(DPM_EHIP);
    }
    int r = 0;
    for (int i = 0; i < ng; ++i) { rk[i] = r; r += fl[i]; }
    // first gamma_in row of each z-plane (the lists ascend in linear index)
    {
      std::vector<int32_t> ix(ng), zo(g.n + 1, 0);
      if (hipMemcpy(ix.data(), b->idx, sizeof(int32_t) * ng, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("dpm_build_boundary_matrix: copy failed");
        return fail(DPM_EHIP);
      }
      const long long nn = (long long)g.n * g.n;
      for (int i = 0; i < ng; ++i)
        if (fl[i]) ++zo[(int)(ix[i] / nn) + 1];
      for (int z = 0; z < g.n; ++z) zo[z + 1] += zo[z];
      if (hipMemcpy(b->in_zoff, zo.data(), sizeof(int32_t) * (g.n + 1), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("dpm_build_boundary_matrix: copy failed");
        return fail(DPM_EHIP);
      }
    }
    int32_t* drk = nullptr;
    if (hipMalloc(&drk, sizeof(int32_t) * ng) != hipSuccess) {
      set_error("dpm_build_boundary_matrix: device allocation failed");
      return fail(DPM_ENOMEM);
    }
    hipError_t e = hipMemcpy(drk, rk.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_in_lists, dim3(grid1(ng)), dim3(kB), 0, s, b->idx, b->is_in, drk, ng,
                         b->idx_in, b->pos_in);
      hipLaunchKernelGGL(k_nplus, dim3(4096), dim3(kB), 0, s, b->m_plus, b->idx, ng, b->n_plus, vsz, 0);
      hipLaunchKernelGGL(k_nplus, dim3(grid1(ng)), dim3(kB), 0, s, b->m_plus, b->idx, ng, b->n_plus, vsz, 1);
      hipLaunchKernelGGL(k_gpos, dim3(4096), dim3(kB), 0, s, b->idx, ng, b->gpos, vsz, 0);
      hipLaunchKernelGGL(k_gpos, dim3(grid1(ng)), dim3(kB), 0, s, b->idx, ng, b->gpos, vsz, 1);
      e = hipStreamSynchronize(s);
    }
    (void)hipFree(drk);
    if (e != hipSuccess) {
      set_error("dpm_build_boundary_matrix: %s", hipGetErrorString(e));
      return fail(DPM_EHIP);
    }
  }
  {
    // Step 2 creates the handle: its build scratch is allocated here and freed after the build
    // (rebuilds take theirs from the caller)
    const size_t sb = factor ? rebuild_scratch_bytes(b) : columns_scratch_bytes(b);
    void* scratch = nullptr;
    if (hipMalloc(&scratch, sb) != hipSuccess) {
      set_error("dpm_build_boundary_matrix: device allocation of %zu scratch bytes failed", sb);
      return fail(DPM_ENOMEM);
    }
    dpm_status st = factor ? factor_bep(b, s, A_out, scratch, sb) : bep_columns(b, s, scratch, sb);
    const hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(scratch);
    if (st == DPM_OK && e != hipSuccess) {
      set_error("dpm_build_boundary_matrix: %s", hipGetErrorString(e));
      st = DPM_EHIP;
    }
    if (st != DPM_OK) return fail(st);
  }
  *out = b;
  return DPM_OK;
}

dpm_status rebuild_bep_impl(dpm_bep* b, double sigma, hipStream_t s, void* scratch,
                            size_t bytes) {
  if (scratch == nullptr || bytes < rebuild_scratch_bytes(b)) {
    set_error("dpm_bep_rebuild: workspace too small: %zu bytes given, %zu needed", bytes,
              rebuild_scratch_bytes(b));
    return DPM_EINVAL;
  }
  b->grid.sigma = sigma;
  return factor_bep(b, s, nullptr, scratch, bytes);
}

void destroy_bep(dpm_bep* b) {
  if (!b) return;
  (void)hipFree(b->m_plus);
  (void)hipFree(b->n_plus);
  (void)hipFree(b->idx);
  (void)hipFree(b->is_in);
  (void)hipFree(b->idx_in);
  (void)hipFree(b->pos_in);
  (void)hipFree(b->in_zoff);
  (void)hipFree(b->basis);
  (void)hipFree(b->A);
  (void)hipFree(b->tau);
  (void)hipFree(b->P);
  (void)hipFree(b->gpos);
  delete b;
}

}  // namespace dpm
