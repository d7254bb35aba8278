// Truncated minimum-norm least squares for a numerically rank-deficient boundary matrix.
//
// After the Householder QR A = Q R (bep.hip), the least-squares operator is P = R+ Q1^T with R+
// the pseudo-inverse of the n x n triangle R truncated at rcond: the singular values of R (those
// of A) below rcond * s_max are taken as zero.  The SVD of R is computed by one-sided Jacobi
// (Hestenes): W = R V is orthogonalised column pair by column pair, V accumulating the plane
// rotations, until every pair is orthogonal to a relative 1e-14; then W = U diag(s),
// s_i = ||w_i||, and R+ = V diag(1/s) U^T = sum over kept i of v_i w_i^T / s_i^2.
//
// Parallel order (block Jacobi): the padded columns form nb blocks of BS; a launch pairs the
// blocks round-robin (nb/2 pairs, one workgroup each), and a workgroup loads its two blocks of W
// and V into LDS and sweeps every pair of its 2 BS columns round-robin (BS pairs at a time).
// nb - 1 launches make one sweep over all column pairs.  The number of launches is fixed (no host
// synchronisation): after each sweep a one-thread kernel raises a flag once the sweep's largest
// pair cosine is below the tolerance, and later launches exit at entry.
#include <cmath>

#include "bep.h"

namespace dpm {

namespace {

constexpr int kST = 256;           // threads of a pair-sweep workgroup
constexpr double kRotTol = 1e-15;  // rotate a pair whose cosine exceeds this
constexpr double kConvTol = 1e-14; // a sweep whose largest cosine is below this ends the SVD
constexpr int kMaxSweeps = 32;

// flags[0]: largest pair cosine of the running sweep (bit pattern of a non-negative double),
// flags[1]: converged (set once, read by every later launch), flags[2]: squared norm below which
// a column is negligible (bit pattern): rcond^2 ||R||_F^2 / (100 n) <= (rcond s_max / 10)^2, so
// such a column stays below the truncation; a pair of two negligible columns is neither rotated
// nor counted for convergence (their mutual angle does not enter the truncated pseudo-inverse).
__global__ __launch_bounds__(1024) void k_svd_neg(const double* __restrict__ A, int m, int n,
                                                  double rcond,
                                                  unsigned long long* __restrict__ flags) {
  __shared__ double red[16];
  double s = 0.0;
  for (long long e = threadIdx.x; e < (long long)n * n; e += 1024) {
    const int c = (int)(e / n), r = (int)(e - (long long)c * n);
    if (r <= c) {
      const double v = A[(long long)c * m + r];
      s += v * v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    flags[2] = (unsigned long long)__double_as_longlong(rcond * rcond * t / (100.0 * n));
  }
}

__global__ void k_svd_init(const double* __restrict__ A, int m, int n, int np,
                           double* __restrict__ W, double* __restrict__ V,
                           unsigned long long* __restrict__ flags) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) { flags[0] = 0ull; flags[1] = 0ull; }
  if (e >= (long long)np * np) return;
  const int c = (int)(e / np), r = (int)(e - (long long)c * np);  // column-major (row r, column c)
  W[e] = (r <= c && c < n) ? A[(long long)c * m + r] : 0.0;      // the upper triangle R
  V[e] = r == c ? 1.0 : 0.0;
}

// Round-robin partner of player k in round r among P players (P even): the pairs of a round are
// disjoint and the P - 1 rounds meet every pair once.
__device__ __forceinline__ void rr_pair(int r, int k, int P, int& a, int& b) {
  const int q = P - 1;
  if (k == 0) {
    a = r % q;
    b = q;
  } else {
    a = (r + k) % q;
    b = (r - k + q) % q;
  }
}

// LDS of a pair-sweep workgroup: W then V columns of its two blocks, [2 BS][np] each; the
// padded size np is at most kSvdLds / (4 BS) (320 columns at BS = 16, 640 at BS = 8).
constexpr int kSvdLds = 20480;  // doubles: the CU's 160 KB

template <int BS>
__global__ __launch_bounds__(kST) void k_svd_round(double* __restrict__ W, double* __restrict__ V,
                                                   int np, int nb, int round,
                                                   unsigned long long* __restrict__ flags) {
  __shared__ double sm[kSvdLds];
  if (flags[1] != 0ull) return;   // converged in an earlier sweep: uniform exit
  const double neg2 = __longlong_as_double((long long)flags[2]);
  constexpr int C2 = 2 * BS;      // columns held
  constexpr int TPP = kST / BS;   // threads per column pair
  double* wl = sm;
  double* vl = sm + (size_t)C2 * np;
  int bi, bj;
  rr_pair(round, blockIdx.x, nb, bi, bj);
  const int t = threadIdx.x;
  // load: local column c < BS is global column bi*BS + c, c >= BS is bj*BS + (c - BS)
  for (int e = t; e < C2 * np; e += kST) {
    const int c = e / np, r = e - c * np;
    const int gc = c < BS ? bi * BS + c : bj * BS + (c - BS);
    wl[e] = W[(long long)gc * np + r];
    vl[e] = V[(long long)gc * np + r];
  }
  __syncthreads();
  const int pr = t / TPP, lt = t % TPP;  // pair of this thread, lane within the pair
  double cmax = 0.0;
  for (int rr = 0; rr < C2 - 1; ++rr) {
    int p, q;
    rr_pair(rr, pr, C2, p, q);
    double* wp = wl + (size_t)p * np;
    double* wq = wl + (size_t)q * np;
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = lt; i < np; i += TPP) {
      const double x = wp[i], y = wq[i];
      al += x * x;
      be += y * y;
      ga += x * y;
    }
    for (int off = TPP / 2; off > 0; off >>= 1) {  // fixed butterfly within the pair's lanes
      al += __shfl_xor(al, off, TPP);
      be += __shfl_xor(be, off, TPP);
      ga += __shfl_xor(ga, off, TPP);
    }
    if (al > 0.0 && be > 0.0 && fmax(al, be) >= neg2) {
      const double cosv = fabs(ga) / sqrt(al * be);
      cmax = fmax(cmax, cosv);
      if (cosv > kRotTol) {
        // rotation zeroing the pair's off-diagonal Gram entry (the root of smaller magnitude)
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        double* vp = vl + (size_t)p * np;
        double* vq = vl + (size_t)q * np;
        for (int i = lt; i < np; i += TPP) {
          const double x = wp[i], y = wq[i];
          wp[i] = cs * x - sn * y;
          wq[i] = sn * x + cs * y;
          const double u = vp[i], w = vq[i];
          vp[i] = cs * u - sn * w;
          vq[i] = sn * u + cs * w;
        }
      }
    }
    __syncthreads();
  }
  for (int e = t; e < C2 * np; e += kST) {
    const int c = e / np, r = e - c * np;
    const int gc = c < BS ? bi * BS + c : bj * BS + (c - BS);
    W[(long long)gc * np + r] = wl[e];
    V[(long long)gc * np + r] = vl[e];
  }
  // largest cosine of this workgroup -> the sweep's maximum (order independent)
  for (int off = 32; off > 0; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
  if ((t & 63) == 0) atomicMax(flags, (unsigned long long)__double_as_longlong(cmax));
}

// End of a sweep: converged once its largest cosine is below the tolerance; reset the maximum.
__global__ void k_svd_sweep_end(unsigned long long* __restrict__ flags) {
  if (flags[1] != 0ull) return;
  if (__longlong_as_double((long long)flags[0]) < kConvTol) flags[1] = 1ull;
  flags[0] = 0ull;
}

// s_i^2 = ||w_i||^2; kept iff s_i > rcond s_max; inv[i] = 1/s_i^2 for kept columns, else 0.
// rd[2] = number kept (the numerical rank), rd[3] = smallest kept s / s_max.  One block.
__global__ __launch_bounds__(1024) void k_svd_sigma(const double* __restrict__ W, int n, int np,
                                                    double rcond, double* __restrict__ inv,
                                                    double* __restrict__ rd) {
  __shared__ double red[16];
  const int t = threadIdx.x;
  double mx = 0.0;
  for (int i = t; i < n; i += 1024) {
    double a = 0.0;
    const double* w = W + (long long)i * np;
    for (int r = 0; r < np; ++r) a += w[r] * w[r];
    inv[i] = a;
    mx = fmax(mx, a);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((t & 63) == 0) red[t >> 6] = mx;
  __syncthreads();
  if (t == 0) {
    double m2 = 0.0;
    for (int w = 0; w < 16; ++w) m2 = fmax(m2, red[w]);
    red[0] = m2;
  }
  __syncthreads();
  const double smax2 = red[0];
  const double thr2 = rcond * rcond * smax2;
  __syncthreads();
  int kept = 0;
  double smin2 = smax2;
  for (int i = t; i < n; i += 1024) {
    const double a = inv[i];
    const bool k = a > thr2 && a > 0.0;
    inv[i] = k ? 1.0 / a : 0.0;
    kept += k ? 1 : 0;
    if (k) smin2 = fmin(smin2, a);
  }
  for (int off = 32; off > 0; off >>= 1) {
    kept += __shfl_xor(kept, off);
    smin2 = fmin(smin2, __shfl_xor(smin2, off));
  }
  __shared__ int rk[16];
  __shared__ double rm[16];
  if ((t & 63) == 0) { rk[t >> 6] = kept; rm[t >> 6] = smin2; }
  __syncthreads();
  if (t == 0) {
    int k = 0;
    double m = smax2;
    for (int w = 0; w < 16; ++w) { k += rk[w]; m = fmin(m, rm[w]); }
    rd[2] = (double)k;
    rd[3] = smax2 > 0.0 ? sqrt(m / smax2) : 0.0;
  }
}

// R+[nu][a] = sum_i V[nu][i] W[a][i] inv[i] (row-major n x n).  One thread per entry.
__global__ void k_svd_pinv(const double* __restrict__ W, const double* __restrict__ V,
                           const double* __restrict__ inv, int n, int np,
                           double* __restrict__ Rp) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int nu = e / n, a = e - nu * n;
  double d = 0.0;
  for (int i = 0; i < n; ++i) d += V[(long long)i * np + nu] * W[(long long)i * np + a] * inv[i];
  Rp[e] = d;
}

// K = Rp Wy (general n x n products, row-major).  One thread per entry.
__global__ void k_kmat_full(const double* __restrict__ Rp, const double* __restrict__ Wy, int n,
                            double* __restrict__ K) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int nu = e / n, b = e - nu * n;
  double d = 0.0;
  for (int a = 0; a < n; ++a) d += Rp[(long long)nu * n + a] * Wy[(long long)a * n + b];
  K[e] = d;
}

}  // namespace

SvdShape svd_shape(int n) {
  SvdShape sh{};
  sh.bs = 16;
  int np = (n + 2 * sh.bs - 1) / (2 * sh.bs) * (2 * sh.bs);
  if (4 * sh.bs * np > kSvdLds) {
    sh.bs = 8;
    np = (n + 2 * sh.bs - 1) / (2 * sh.bs) * (2 * sh.bs);
  }
  sh.np = np;
  sh.nb = np / sh.bs;
  sh.ok = 4 * sh.bs * np <= kSvdLds;
  return sh;
}

dpm_status pinv_of_r(const double* A, int m, int n, double rcond, double* Rp, double* W,
                     double* V, double* inv, unsigned long long* flags, double* rd,
                     hipStream_t s) {
  const SvdShape sh = svd_shape(n);
  if (!sh.ok) {
    set_error("truncated least squares: %d columns exceed the Jacobi SVD's limit", n);
    return DPM_EINVAL;
  }
  const long long nn = (long long)sh.np * sh.np;
  hipLaunchKernelGGL(k_svd_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, m, n,
                     sh.np, W, V, flags);
  hipLaunchKernelGGL(k_svd_neg, dim3(1), dim3(1024), 0, s, A, m, n, rcond, flags);
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    for (int r = 0; r < sh.nb - 1; ++r) {
      if (sh.bs == 16)
        hipLaunchKernelGGL(k_svd_round<16>, dim3(sh.nb / 2), dim3(kST), 0, s, W, V, sh.np,
                           sh.nb, r, flags);
      else
        hipLaunchKernelGGL(k_svd_round<8>, dim3(sh.nb / 2), dim3(kST), 0, s, W, V, sh.np,
                           sh.nb, r, flags);
    }
    hipLaunchKernelGGL(k_svd_sweep_end, dim3(1), dim3(1), 0, s, flags);
  }
  hipLaunchKernelGGL(k_svd_sigma, dim3(1), dim3(1024), 0, s, W, n, sh.np, rcond, inv, rd);
  hipLaunchKernelGGL(k_svd_pinv, dim3((unsigned)(((long long)n * n + 255) / 256)), dim3(256), 0,
                     s, W, V, inv, n, sh.np, Rp);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

void kmat_full(const double* Rp, const double* Wy, int n, double* K, hipStream_t s) {
  hipLaunchKernelGGL(k_kmat_full, dim3((unsigned)(((long long)n * n + 255) / 256)), dim3(256), 0,
                     s, Rp, Wy, n, K);
}

}  // namespace dpm
