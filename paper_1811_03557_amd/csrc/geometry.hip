// Geometry of the DPM on the device: the M+ mask, the discrete grid boundary gamma and the
// spectral densities of the extension operator (paper Sec. 2: Def. "point sets", eqs
// extension_operator1, spectral_approximation_sd, extension_operator_recast).
#include <cmath>
#include <vector>

#include "common.h"
#include "geom_dev.h"

namespace dpm {

dpm_status validate_geometry(const dpm_geometry* geo) {
  if (!geo) { set_error("geometry is NULL"); return DPM_EINVAL; }
  if (geo->kind != 0 && geo->kind != 1) { set_error("geometry kind must be 0 (sphere) or 1 (ellipsoid)"); return DPM_EINVAL; }
  const int na = geo->kind == 0 ? 1 : 3;
  for (int i = 0; i < na; ++i)
    if (!(geo->axes[i] > 0.0) || !std::isfinite(geo->axes[i])) { set_error("axes must be finite and > 0"); return DPM_EINVAL; }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(geo->center[i])) { set_error("center must be finite"); return DPM_EINVAL; }
  return DPM_OK;
}

namespace {

__global__ void k_classify(int n, double h, double x0, GeoDev g, uint8_t* __restrict__ m) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long vol = (long long)n * n * n;
  if (i >= vol) return;
  const int ix = (int)(i % n);
  const int iy = (int)((i / n) % n);
  const int iz = (int)(i / ((long long)n * n));
  m[i] = inside(g, x0 + h * ix, x0 + h * iy, x0 + h * iz) ? 1 : 0;
}

constexpr int kGBlock = 256;
constexpr int kGItems = 8;  // nodes per thread: a block covers 2048 consecutive nodes

// flags of node i: bit 0 = gamma, bit 1 = gamma_in; sets *bad when an M+ node touches the
// ghost layer (N+ would leave M0).
__device__ __forceinline__ int gamma_flags(const uint8_t* __restrict__ m, int n, long long i,
                                           int* bad) {
  const int ix = (int)(i % n);
  const int iy = (int)((i / n) % n);
  const int iz = (int)(i / ((long long)n * n));
  const bool plus = m[i] != 0;
  const bool edge = ix == 0 || iy == 0 || iz == 0 || ix == n - 1 || iy == n - 1 || iz == n - 1;
  if (plus && edge) atomicOr(bad, 1);
  bool nb_plus = false, nb_minus = false;
  const long long nn = (long long)n * n;
  if (ix > 0) { bool q = m[i - 1] != 0; nb_plus |= q; nb_minus |= !q; }
  if (ix < n - 1) { bool q = m[i + 1] != 0; nb_plus |= q; nb_minus |= !q; }
  if (iy > 0) { bool q = m[i - n] != 0; nb_plus |= q; nb_minus |= !q; }
  if (iy < n - 1) { bool q = m[i + n] != 0; nb_plus |= q; nb_minus |= !q; }
  if (iz > 0) { bool q = m[i - nn] != 0; nb_plus |= q; nb_minus |= !q; }
  if (iz < n - 1) { bool q = m[i + nn] != 0; nb_plus |= q; nb_minus |= !q; }
  // node in N+ : in M+ or next to M+; in N- : in M- or next to M-
  const bool in_np = plus || nb_plus;
  const bool in_nm = !plus || nb_minus;
  const bool gam = in_np && in_nm;
  return gam ? (plus ? 3 : 1) : 0;
}

// Pass 1: per-block counts of gamma and gamma_in.  Pass 2: ordered compaction.
__global__ __launch_bounds__(kGBlock) void k_gamma(const uint8_t* __restrict__ m, int n,
                                                   int* __restrict__ counts,      // [2][blocks]
                                                   const int* __restrict__ offs,  // nullable
                                                   int32_t* __restrict__ idx,
                                                   uint8_t* __restrict__ is_in, int* bad) {
  __shared__ int scan[kGBlock];
  const long long vol = (long long)n * n * n;
  const long long start = (long long)blockIdx.x * kGBlock * kGItems + (long long)threadIdx.x * kGItems;
  int fl[kGItems];
  int cnt = 0, cnt_in = 0;
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    const long long i = start + k;
    fl[k] = (i < vol) ? gamma_flags(m, n, i, bad) : 0;
    cnt += fl[k] & 1;
    cnt_in += (fl[k] >> 1) & 1;
  }
  if (offs == nullptr) {
    // block sums
    scan[threadIdx.x] = cnt | (cnt_in << 16);
    __syncthreads();
    for (int off = kGBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) scan[threadIdx.x] += scan[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      counts[blockIdx.x] = scan[0] & 0xffff;
      counts[gridDim.x + blockIdx.x] = scan[0] >> 16;
    }
    return;
  }
  // inclusive Hillis-Steele scan of the per-thread counts
  scan[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < kGBlock; off <<= 1) {
    int v = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  int o = offs[blockIdx.x] + scan[threadIdx.x] - cnt;
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    if (fl[k] & 1) {
      idx[o] = (int32_t)(start + k);
      is_in[o] = (uint8_t)((fl[k] >> 1) & 1);
      ++o;
    }
  }
}

// Real orthonormal spherical harmonics, no Condon-Shortley phase, through the normalised
// associated Legendre functions Pbar_l^m (integral of Pbar^2 over the sphere with the azimuthal
// factor equal to 1):
//   Pbar_0^0 = 1/sqrt(4 pi),  Pbar_m^m = sqrt((2m+1)/(2m)) sin(theta) Pbar_{m-1}^{m-1},
//   Pbar_{m+1}^m = sqrt(2m+3) cos(theta) Pbar_m^m,
//   Pbar_l^m = sqrt((4l^2-1)/(l^2-m^2)) (cos(theta) Pbar_{l-1}^m
//              - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) Pbar_{l-2}^m);
//   Y_l0 = Pbar_l^0, Y_lm = sqrt(2) Pbar_l^m cos(m phi), Y_l,-m = sqrt(2) Pbar_l^m sin(m phi).
__global__ void k_basis(int n, double h, double x0, GeoDev g, int ng,
                        const int32_t* __restrict__ idx, int lmax, int beta,
                        double* __restrict__ basis, double* __restrict__ d_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const long long li = idx[i];
  const int ix = (int)(li % n);
  const int iy = (int)((li / n) % n);
  const int iz = (int)(li / ((long long)n * n));
  double d, th, ph;
  project(g, x0 + h * ix - g.cx, x0 + h * iy - g.cy, x0 + h * iz - g.cz, &d, &th, &ph);
  if (d_out) d_out[i] = d;
  const int nlm = (lmax + 1) * (lmax + 1);
  const double ct = cos(th), st = sin(th);
  const double half_d2 = 0.5 * d * d;
  const double rt2 = 1.4142135623730950488;
  double pmm = 0.28209479177387814347;  // 1/sqrt(4 pi)
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) pmm *= sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
    double cm = 1.0, sm = 0.0;
    if (m > 0) sincos(m * ph, &sm, &cm);
    double p_lm2 = 0.0, p_lm1 = pmm;
    for (int l = m; l <= lmax; ++l) {
      double p;
      if (l == m) {
        p = pmm;
      } else if (l == m + 1) {
        p = sqrt(2.0 * m + 3.0) * ct * pmm;
        p_lm2 = pmm;
        p_lm1 = p;
      } else {
        const double al = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double bl = sqrt(((double)(l - 1) * (l - 1) - (double)m * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
        p = al * (ct * p_lm1 - bl * p_lm2);
        p_lm2 = p_lm1;
        p_lm1 = p;
      }
      const int base = l * l + l;  // index of (l, 0)
      if (m == 0) {
        basis[(long long)base * ng + i] = p;
        if (beta) basis[(long long)(nlm + base) * ng + i] = half_d2 * p;
      } else {
        const double yc = rt2 * p * cm, ys = rt2 * p * sm;
        basis[(long long)(base + m) * ng + i] = yc;
        basis[(long long)(base - m) * ng + i] = ys;
        if (beta) {
          basis[(long long)(nlm + base + m) * ng + i] = half_d2 * yc;
          basis[(long long)(nlm + base - m) * ng + i] = half_d2 * ys;
        }
      }
    }
  }
}

// Zonal densities: P_nu(cos theta) (Legendre, unnormalised), nu = 0..mmax, by the three-term
// recurrence (nu + 1) P_{nu+1} = (2 nu + 1) x P_nu - nu P_{nu-1}, stable for |x| <= 1; rows
// mmax + 1 .. carry (d^2/2) P_nu when beta = 1.
__global__ void k_basis_zonal(int n, double h, double x0, GeoDev g, int ng,
                              const int32_t* __restrict__ idx, int mmax, int beta,
                              double* __restrict__ basis, double* __restrict__ d_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const long long li = idx[i];
  const int ix = (int)(li % n);
  const int iy = (int)((li / n) % n);
  const int iz = (int)(li / ((long long)n * n));
  double d, th, ph;
  project(g, x0 + h * ix - g.cx, x0 + h * iy - g.cy, x0 + h * iz - g.cz, &d, &th, &ph);
  if (d_out) d_out[i] = d;
  const double x = cos(th), half_d2 = 0.5 * d * d;
  const long long off2 = (long long)(mmax + 1) * ng;
  double pm1 = 0.0, p = 1.0;  // P_{nu-1}, P_nu
  for (int nu = 0; nu <= mmax; ++nu) {
    basis[(long long)nu * ng + i] = p;
    if (beta) basis[off2 + (long long)nu * ng + i] = half_d2 * p;
    const double pn = ((2.0 * nu + 1.0) * x * p - nu * pm1) / (nu + 1.0);
    pm1 = p;
    p = pn;
  }
}

}  // namespace

dpm_status classify_impl(const dpm_grid& g, const dpm_geometry& geo, uint8_t* m_plus, hipStream_t s) {
  const long long vol = (long long)g.n * g.n * g.n;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((vol + 255) / 256)), dim3(256), 0, s, g.n, g.h,
                     g.x0, to_dev(geo), m_plus);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

dpm_status gamma_points_impl(const dpm_grid& g, const uint8_t* m_plus, int32_t* n_gamma,
                             int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, hipStream_t s) {
  const long long vol = (long long)g.n * g.n * g.n;
  const int blocks = (int)((vol + kGBlock * kGItems - 1) / (kGBlock * kGItems));
  int* dcounts = nullptr;
  int* doffs = nullptr;
  int* dbad = nullptr;
  dpm_status st = DPM_OK;
  std::vector<int> counts(2 * (size_t)blocks), offs(blocks);
  int bad = 0;
  long long tot = 0, tot_in = 0;
  auto cleanup = [&]() {
    (void)hipFree(dcounts);
    (void)hipFree(doffs);
    (void)hipFree(dbad);
  };
  if (hipMalloc(&dcounts, sizeof(int) * 2 * blocks) != hipSuccess ||
      hipMalloc(&doffs, sizeof(int) * blocks) != hipSuccess ||
      hipMalloc(&dbad, sizeof(int)) != hipSuccess) {
    cleanup();
    set_error("gamma_points: device allocation failed");
    return DPM_ENOMEM;
  }
  hipError_t e = hipMemsetAsync(dbad, 0, sizeof(int), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gamma, dim3(blocks), dim3(kGBlock), 0, s, m_plus, g.n, dcounts,
                       (const int*)nullptr, (int32_t*)nullptr, (uint8_t*)nullptr, dbad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(counts.data(), dcounts, sizeof(int) * 2 * blocks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    set_error("gamma_points: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  for (int b = 0; b < blocks; ++b) {
    offs[b] = (int)tot;
    tot += counts[b];
    tot_in += counts[blocks + b];
  }
  if (bad) {
    cleanup();
    set_error("geometry touches the ghost layer: M+ has nodes on the outermost interior layer");
    return DPM_EGEOM;
  }
  if (tot == 0) {
    cleanup();
    set_error("gamma is empty");
    return DPM_EGEOM;
  }
  *n_gamma = (int32_t)tot;
  *n_gamma_in = (int32_t)tot_in;
  if (idx != nullptr) {
    e = hipMemcpyAsync(doffs, offs.data(), sizeof(int) * blocks, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_gamma, dim3(blocks), dim3(kGBlock), 0, s, m_plus, g.n, dcounts,
                         (const int*)doffs, idx, is_in, dbad);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      cleanup();
      set_error("gamma_points: %s", hipGetErrorString(e));
      return DPM_EHIP;
    }
  }
  cleanup();
  return st;
}

dpm_status basis_impl(const dpm_grid& g, const dpm_geometry& geo, int32_t n_gamma,
                      const int32_t* idx, int32_t lmax, int32_t beta, double* basis, double* d_out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_basis, dim3((n_gamma + 127) / 128), dim3(128), 0, s, g.n, g.h, g.x0,
                     to_dev(geo), n_gamma, idx, lmax, beta, basis, d_out);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

dpm_status basis_zonal_impl(const dpm_grid& g, const dpm_geometry& geo, int32_t n_gamma,
                            const int32_t* idx, int32_t mmax, int32_t beta, double* basis,
                            double* d_out, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_zonal, dim3((n_gamma + 127) / 128), dim3(128), 0, s, g.n, g.h, g.x0,
                     to_dev(geo), n_gamma, idx, mmax, beta, basis, d_out);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace dpm
