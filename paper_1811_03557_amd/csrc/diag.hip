// The quantities tracked along a run (paper Sec. 4, "Error metrics and quantities of interest"):
// max |rho| over M+, the second moment sum_{M+} h^3 |x|^2 rho, and the free energy
// sum_{M+} h^3 (rho ln rho - rho c + c^2/2 + (1/(8h^2)) sum_axes (c_{+1} - c_{-1})^2), for one
// domain or summed over the two subdomains of the domain decomposition (maximum over both).
// rho ln rho is 0 for rho <= 0 (its limit at 0: the scheme keeps rho >= 0 up to rounding); a NaN
// rho makes the free energy and the maximum NaN.
//
// Deterministic: every block reduces its grid-stride share in a fixed order into partials, and
// one block adds the partials in a fixed order (no atomics), so a result is reproducible bitwise.
#include <cmath>

#include "bep.h"

namespace dpm {

const dpm_bep* dd_sub(const dpm_dd* d, int l);
const double* dd_origin(const dpm_dd* d, int l);

namespace {

constexpr int kT = 256;
constexpr int kParts = 512;  // blocks of the partial pass (per domain)

// NaN-propagating maximum
__device__ __forceinline__ double nmax(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ __forceinline__ void block_reduce3(double& mx, double& s1, double& s2, double* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    mx = nmax(mx, __shfl_down(mx, o));
    s1 += __shfl_down(s1, o);
    s2 += __shfl_down(s2, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[3 * wave] = mx;
    sh[3 * wave + 1] = s1;
    sh[3 * wave + 2] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kT / 64; ++w) {
      mx = nmax(mx, sh[3 * w]);
      s1 += sh[3 * w + 1];
      s2 += sh[3 * w + 2];
    }
  }
}

__global__ __launch_bounds__(kT) void k_diag_part(const double* __restrict__ rho,
                                                  const double* __restrict__ c,
                                                  const uint8_t* __restrict__ mp, int n, double h,
                                                  double x0, double ox, double oy, double oz,
                                                  double* __restrict__ part) {
  __shared__ double sh[3 * (kT / 64)];
  const long long vol = (long long)n * n * n, nn = (long long)n * n;
  const double h3 = h * h * h, i8h2 = 1.0 / (8.0 * h * h);
  double mx = 0.0, m2 = 0.0, fe = 0.0;
  for (long long i = (long long)blockIdx.x * kT + threadIdx.x; i < vol;
       i += (long long)gridDim.x * kT) {
    if (!mp[i]) continue;
    const int ix = (int)(i % n);
    const int iy = (int)((i / n) % n);
    const int iz = (int)(i / nn);
    const double X = x0 + h * ix + ox, Y = x0 + h * iy + oy, Z = x0 + h * iz + oz;
    const double r = rho[i], cc = c[i];
    mx = nmax(mx, fabs(r));
    m2 += h3 * (X * X + Y * Y + Z * Z) * r;
    // M+ nodes have all six neighbours inside the cube (N+ does not reach the ghost layer)
    const double gx = c[i + 1] - c[i - 1], gy = c[i + n] - c[i - n], gz = c[i + nn] - c[i - nn];
    const double rlr = r > 0.0 ? r * log(r) : (r != r ? r : 0.0);
    fe += h3 * (rlr - r * cc + 0.5 * cc * cc + (gx * gx + gy * gy + gz * gz) * i8h2);
  }
  block_reduce3(mx, m2, fe, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = mx;
    part[3 * blockIdx.x + 1] = m2;
    part[3 * blockIdx.x + 2] = fe;
  }
}

// out3 = (max, sum, sum) over nparts partials, each thread taking a strided share in order
__global__ __launch_bounds__(kT) void k_diag_final(const double* __restrict__ part, int nparts,
                                                   double* __restrict__ out3) {
  __shared__ double sh[3 * (kT / 64)];
  double mx = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kT) {
    mx = nmax(mx, part[3 * k]);
    s1 += part[3 * k + 1];
    s2 += part[3 * k + 2];
  }
  block_reduce3(mx, s1, s2, sh);
  if (threadIdx.x == 0) {
    out3[0] = mx;
    out3[1] = s1;
    out3[2] = s2;
  }
}

unsigned part_blocks(long long vol) {
  const long long b = (vol + kT - 1) / kT;
  return (unsigned)(b < kParts ? b : kParts);
}

void launch_part(const dpm_bep* b, const double* origin, const double* rho, const double* c,
                 double* part, hipStream_t s) {
  const dpm_grid& g = b->grid;
  const long long vol = (long long)g.n * g.n * g.n;
  hipLaunchKernelGGL(k_diag_part, dim3(part_blocks(vol)), dim3(kT), 0, s, rho, c, b->m_plus, g.n,
                     g.h, g.x0, origin[0], origin[1], origin[2], part);
}

}  // namespace

size_t diag_workspace_bytes() { return sizeof(double) * 3 * 2 * kParts; }

dpm_status diagnostics_impl(const dpm_bep* b, const double* rho, const double* c, double* out3,
                            void* ws, hipStream_t s) {
  const double zero[3] = {0.0, 0.0, 0.0};
  double* part = static_cast<double*>(ws);
  const dpm_grid& g = b->grid;
  launch_part(b, zero, rho, c, part, s);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kT), 0, s, part,
                     (int)part_blocks((long long)g.n * g.n * g.n), out3);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

dpm_status dd_diagnostics_impl(const dpm_dd* d, const double* const state[4], double* out3,
                               void* ws, hipStream_t s) {
  double* part = static_cast<double*>(ws);
  int off = 0;
  for (int l = 0; l < 2; ++l) {
    const dpm_bep* b = dd_sub(d, l);
    launch_part(b, dd_origin(d, l), state[2 * l], state[2 * l + 1], part + 3 * off, s);
    off += (int)part_blocks((long long)b->grid.n * b->grid.n * b->grid.n);
  }
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kT), 0, s, part, off, out3);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace dpm
