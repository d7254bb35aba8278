// Middle pass of the auxiliary-problem solve: a tridiagonal solve along z in the (kx, ky)
// eigenbasis (Fourier analysis in x and y, elimination in z: Hockney's fast Poisson solver).
//
// After the forward DST-Is along x and y, the spectral column (kx, ky) of the volume obeys the
// one-dimensional AP along z with zero Dirichlet ends.  Times h^2 it reads
//   -u_{z-1} + (2 + eps) u_z - u_{z+1} = h^2 f_z,   eps = h^2 sigma + lam_hat_kx + lam_hat_ky > 0,
// lam_hat_k = 4 sin^2(pi k / (2(N+1))).  Its exact solution equals the forward DST along z,
// the division by sigma + lambda_kx + lambda_ky + lambda_kz and the inverse DST along z, which
// this pass replaces: the HBM traffic is the same (one read and one write per point), the
// arithmetic is about 25 FP64 operations per point with no LDS shuffles, against two line
// transforms.
//
// Accuracy.  The matrix is near-singular for the low modes (eps down to ~1e-4 at N = 255), and
// forming the diagonal 2 + eps rounds away the part of eps that sets the smallest eigenvalue:
// plain elimination then loses a factor ~1/eps against the DST form.  Every pivot is therefore
// computed from eps alone, as a sum of positive terms.  For tridiag(-1, 2 + eps, -1) the pivots
// are m_k = 1 + t_k with t_1 = 1 + eps, t_k = eps + t_{k-1}/(1 + t_{k-1}).  For a general
// symmetric tridiagonal M-matrix with diagonal d_j, off-diagonals -e_j and row excess
// rho_j = d_j - e_{j-1} - e_j >= 0, the pivots are m_j = e_j + tau_j with
// tau_j = rho_j + e_{j-1} tau_{j-1} / m_{j-1}; the reduced system below uses this form, with
// each rho_j itself a sum of positive terms.  The result matches the DST form's error (a few
// 1e-15 relative at N = 255 ... 1023 in FP64).
//
// Parallel layout.  Each column is cut into segments of 16 rows: 15 unknowns and a separator
// after them (the last segment has no separator; when 16 does not divide n + 1, the first
// segment is short, padded with virtual rows above z = 0).  A block
// owns W adjacent columns (W consecutive elements of every z-plane, so each wavefront load is
// a run of >= 128 contiguous bytes) times all P segments; thread (w, s) holds segment s of
// column w in registers.  Per segment, with T_L = tridiag(-1, 2 + eps, -1) of order L:
//   v = T_L^-1 f_seg, q = T_L^-1 e_L, p = T_L^-1 e_1 (p is q reversed: T_L is persymmetric),
// and the segment's solution is v + z_left p + z_right q for the separator values around it.
// Substituting into the separator rows leaves a symmetric tridiagonal system of P - 1 unknowns:
//   -b z_{j-1} + (2 + eps - a_j - a_{j+1}) z_j - b z_{j+1} = f_sep_j + v_last^j + v_first^{j+1},
// a = q_L = 1/m_L, b = q_1 = prod(1/m_k); its row excesses are eps + (1 - a) at the Dirichlet ends
// and eps + (1 - a - b) per inner segment, with 1 - a = t_L / m_L and
// 1 - a - b = eps * sum_i q_i (both without cancellation).  One thread per column solves it
// from LDS; every thread then reconstructs its rows.  Two block barriers in all.
#include "dst_line.h"

namespace dpm {

namespace {

constexpr int kSegRows = 16;  // rows per segment: 15 unknowns and the separator

// PAD = 16 nseg - 1 - n: the first segment's virtual rows (0 when 16 divides n + 1).
template <typename T, int PAD>
__global__ __launch_bounds__(1024) void k_z_tri(PassArgs p, int n, int nseg, int logw, int tiles,
                                                int nblocks, double fscale) {
  // X[s][w]: separator data of column w (rhs part, then g_j, then z_j); Y[s][w]: v_first of
  // segment s, then 1/m_j
  __shared__ double X[1024], Y[1024];
  const int logical = xcd_remap(blockIdx.x, nblocks);
  const int rhs = logical / tiles;
  const int tile = logical - rhs * tiles;
  if (p.done != nullptr && p.done[p.rhs0 + rhs] != 0) return;  // converged: uniform exit
  const double sig = p.sigma_rhs != nullptr ? p.sigma_rhs[p.rhs0 + rhs] : p.sigma;

  const int tid = threadIdx.x;
  const int W = 1 << logw;
  const int w = tid & (W - 1);
  const int s = tid >> logw;
  const long long plane = (long long)n * n;
  const int col = tile * W + w;
  const bool valid = col < plane;
  const int cc = valid ? col : (int)plane - 1;  // columns past the end reload the last one
  const int r = cc / n;
  const int c = cc - r * n;
  const double h2 = 1.0 / p.inv_h2;
  const double eps = sig * h2 + (p.lam_hat[r] + p.lam_hat[c]);

  // Segment s holds rows z0 .. z0 + 14 and the separator z0 + 15 (the last has none).  With
  // n + 1 = 16 nseg - pad, the rows start pad rows above z = 0: the first segment's first pad
  // rows are virtual (nothing loaded or stored, c = 0 there, so v and q vanish and the pivot
  // recurrence starts at its first real row).
  constexpr bool RAG = PAD != 0;
  constexpr int pad = PAD;
  const bool first = s == 0;
  const bool last = s == nseg - 1;
  const int z0 = s * kSegRows - pad;
  // Wave-uniform base (the first row of the wavefront's first segment, clamped to the volume,
  // and the tile's first column) plus a 32-bit byte offset per lane and row: at most 64 + 15
  // rows of a 1023^2 plane, never negative.
  const int zw0 = ((tid & ~63) >> logw) * kSegRows - pad;
  const int zw = RAG ? max(zw0, 0) : zw0;
  const long long base = (long long)rhs * plane * n + (long long)zw * plane + (long long)tile * W;
  const T* const inb = static_cast<const T*>(p.in) + base;
  T* const outb = static_cast<T*>(p.out) + base;
  const unsigned colb = (unsigned)(cc - tile * W) * (unsigned)sizeof(T);
  const unsigned rowb = (unsigned)plane * (unsigned)sizeof(T);
  // byte offset of local row k (virtual rows read row 0 and are zeroed)
  auto roff = [&](int k) { return colb + (unsigned)((RAG ? max(z0 + k, 0) : z0 + k) - zw) * rowb; };

  // f[0..15): the segment's rows; f[15]: the separator row (zero in the last segment)
  double f[kSegRows];
#pragma unroll
  for (int k = 0; k < kSegRows - 1; ++k) {
    const double v = (double)ld(inb, roff(k));
    f[k] = (!RAG || !first || k >= pad) ? v * fscale : 0.0;
  }
  f[kSegRows - 1] = !last ? (double)ld(inb, roff(kSegRows - 1)) * fscale : 0.0;

  // c_k = 1/m_k (cv[k-1]); 1 - a = t_L/m_L for the full segments and for the first one
  double cv[kSegRows];
  cv[kSegRows - 1] = 0.0;
  double at_full = 0.0, at_first = 1.0;  // an empty first segment: a = 0
  {
    double t = 1.0 + eps;
#pragma unroll
    for (int k = 0; k < kSegRows - 1; ++k) {
      const bool pk = RAG && first && k < pad;
      const double ck = recip(1.0 + t);
      const double tc = t * ck;                   // t_k / m_k = 1 - c_k
      cv[k] = pk ? 0.0 : ck;
      if (k == kSegRows - 2) at_full = tc;
      if (k == kSegRows - 2 - pad) at_first = tc;
      t = pk ? t : eps + tc;
    }
  }

  // v = T_L^-1 f (forward elimination, back substitution), in place
  {
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < kSegRows - 1; ++k) { d = (f[k] + d) * cv[k]; f[k] = d; }
    double vn = 0.0;
#pragma unroll
    for (int k = kSegRows - 2; k >= 0; --k) { vn = f[k] + cv[k] * vn; f[k] = vn; }
  }
  // q = T_L^-1 e_L: suffix products of c, in place of c (p = T_L^-1 e_1 is q reversed for a
  // full segment; the first segment needs no p)
  {
    double qn = 1.0;
#pragma unroll
    for (int k = kSegRows - 2; k >= 0; --k) { qn *= cv[k]; cv[k] = qn; }
  }

  // separator j's right-hand side: f_sep_j + v_last^j (X) + v_first^{j+1} (Y)
  const int ns = nseg - 1;
  if (ns > 0) {
    if (!last) X[s * W + w] = f[kSegRows - 1] + f[kSegRows - 2];
    if (!first) Y[s * W + w] = f[0];
  }
  __syncthreads();

  if (ns > 0 && last) {
    // reduced system of the separators, one thread per column, in the last segment's threads
    // (a full segment: a, b, 1 - a and 1 - a - b of the 15-row segments are its own)
    const double b = cv[0];
    double qs = 0.0;
#pragma unroll
    for (int k = 0; k < kSegRows - 1; ++k) qs += cv[k];
    const double om = eps * qs;
    double tau = 0.0, g = 0.0, im = 0.0;
    for (int j = 0; j < ns; ++j) {
      const bool lsep = j + 1 == ns;
      const double rho = eps + (j == 0 ? at_first : om) + (lsep ? at_full : om);
      const double ej = lsep ? 0.0 : b;
      const double rj = X[j * W + w] + Y[(j + 1) * W + w];
      if (j == 0) { tau = rho; g = rj; }
      else { tau = rho + b * tau * im; g = rj + b * im * g; }
      im = recip(ej + tau);
      X[j * W + w] = g;
      Y[j * W + w] = im;
    }
    double zn = 0.0;
    for (int j = ns - 1; j >= 0; --j) {
      const double ej = j + 1 == ns ? 0.0 : b;
      zn = (X[j * W + w] + ej * zn) * Y[j * W + w];
      X[j * W + w] = zn;
    }
  }
  __syncthreads();

  if (!valid) return;
  // u = v + z_left p + z_right q (z_left = 0 above the first segment, z_right = 0 below the last)
  const double zl = first ? 0.0 : X[(s - 1) * W + w];
  const double zr = last ? 0.0 : X[s * W + w];
#pragma unroll
  for (int k = 0; k < kSegRows - 1; ++k)
    if (!RAG || !first || k >= pad)
      st(outb, roff(k), (T)(f[k] + zl * cv[kSegRows - 2 - k] + zr * cv[k]));
  if (!last) st(outb, roff(kSegRows - 1), (T)zr);
}

// Default columns per block: W * P <= 1024 threads, 16 <= W <= 32 (runs of >= 128 bytes in
// FP64).  At n = 255 (P = 16), W = 32 measured 98.5 us per 2-RHS FP64 launch against 101 at
// W = 64, and 75 against 84 us in FP32; dpm_autotune measures 16, 32 and 64 per size.
int z_tri_logw(int nseg) {
  int logw = 5;
  while (logw > 4 && (nseg << logw) > 1024) --logw;
  return logw;
}

}  // namespace

bool z_tri_supported(int n) { return n >= 1 && n + 1 <= 64 * kSegRows; }

bool z_tri_cols_valid(int n, int cols) {
  const int nseg = (n + kSegRows) / kSegRows;
  return (cols == 16 || cols == 32 || cols == 64) && nseg * cols <= 1024;
}

dpm_status launch_z_tri(int real_bytes, int n, const PassArgs& a, double fscale, int nrhs,
                        hipStream_t s, int cols) {
  if (nrhs <= 0) return DPM_OK;
  if (!z_tri_supported(n)) { set_error("no tridiagonal z pass for n = %d", n); return DPM_EINVAL; }
  const int nseg = (n + kSegRows) / kSegRows;  // ceil((n + 1) / 16)
  if (cols != 0 && !z_tri_cols_valid(n, cols)) {
    set_error("z pass: %d columns per block do not fit n = %d", cols, n);
    return DPM_EINVAL;
  }
  const int logw = cols == 0 ? z_tri_logw(nseg) : (cols == 16 ? 4 : cols == 32 ? 5 : 6);
  const long long plane = (long long)n * n;
  const long long tiles = (plane + (1LL << logw) - 1) >> logw;
  const long long nb = tiles * nrhs;
  if (nb > 0x7fffffffLL) { set_error("launch too large"); return DPM_EINVAL; }
  const dim3 grid((unsigned)nb), block((unsigned)(nseg << logw));
  const int pad = nseg * kSegRows - 1 - n;
  const int ti = (int)tiles, nbi = (int)nb;
  switch (pad) {
#define DPM_ZTRI_CASE(P_)                                                                     \
  case P_:                                                                                    \
    if (real_bytes == 4)                                                                      \
      hipLaunchKernelGGL((k_z_tri<float, P_>), grid, block, 0, s, a, n, nseg, logw, ti, nbi, fscale); \
    else                                                                                      \
      hipLaunchKernelGGL((k_z_tri<double, P_>), grid, block, 0, s, a, n, nseg, logw, ti, nbi, fscale); \
    break;
    DPM_ZTRI_CASE(0) DPM_ZTRI_CASE(1) DPM_ZTRI_CASE(2) DPM_ZTRI_CASE(3) DPM_ZTRI_CASE(4)
    DPM_ZTRI_CASE(5) DPM_ZTRI_CASE(6) DPM_ZTRI_CASE(7) DPM_ZTRI_CASE(8) DPM_ZTRI_CASE(9)
    DPM_ZTRI_CASE(10) DPM_ZTRI_CASE(11) DPM_ZTRI_CASE(12) DPM_ZTRI_CASE(13) DPM_ZTRI_CASE(14)
    DPM_ZTRI_CASE(15)
#undef DPM_ZTRI_CASE
    default: set_error("z pass padding %d", pad); return DPM_EINVAL;
  }
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace dpm
