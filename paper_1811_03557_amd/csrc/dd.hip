// Domain decomposition of the DPM (paper Sec. 3): Case 1 ("Case 1" and "BEPs for Case 1", eqs
// interface_condition, DD1_BEP1, DD1_BEP2, reduced_DD1_BEP1, reduced_DD1_BEP2) and Case 2
// ("Case 2" and "BEPs for Case 2", eqs DD2_BEP, reduced_DD2_BEP, effective densities; below,
// from k_dd2_classify on), one handle type and one step for both, plus the adaptive loop and a
// graph-captured fixed-dt loop on the decomposed domain.
//
// Case 1: Omega_1 = {|x - c| < r_z} (the ball inside the interface sphere Z) and Omega_2 = {r_z < |x - c|
// < r_gamma} (the shell between Z and Gamma), each on its own cube and mesh.  zeta_1 (the discrete
// grid interface of Omega_1) is Omega_1's gamma; Omega_2's gamma is the union of the discrete grid
// boundary near Gamma and zeta_2 near Z, split at the radius r_split.  The densities are zonal
// spectral extensions: near Gamma P_nu and beta (d_G^2/2) P_nu (d_G = |x - c| - r_gamma, zero
// Neumann data); near Z P_nu, d_Z P_nu and (d_Z^2/2) P_nu (d_Z = |x - c| - r_z along the radial
// normal from both sides), whose coefficients are shared by the two subdomains: one coefficient
// set carries the continuity of u and of its first two normal derivatives across Z.  The two
// reduced BEPs are stacked into one least-squares problem, columns [Gamma part ; Z part]:
//
//        [ 0    A_1 ] [C]   [Tr_zeta_1,in G_1 f_1   ]
//        [ A_2^G A_2^Z] [A] = [Tr_gamma_2,in G_2 f_2 ]
//
// (A_l: the reduced-BEP matrix of subdomain l on its own densities), factored once by the FP64
// Householder QR of the single-domain path.  A step solves the particular solutions on both
// meshes, the coupled least squares, and each subdomain's Green's formula.  In Case 2 both
// subdomains carry all columns, wedge nodes add a second row, and each row is mapped to its
// node (row_idx), so the same step serves both cases.
#include <cmath>
#include <vector>

#include "bep.h"

struct dpm_dd {
  dpm_dd_params prm{};
  dpm_bep* sub[2] = {nullptr, nullptr};  // per subdomain: masks, gamma lists, densities, A_l
  int n_gamma_cols = 0, n_z_cols = 0, n_cols = 0;
  int rows = 0;           // reduced-BEP rows of both subdomains (Case 1: |zeta_1,in| + |gamma_2,in|)
  double* A = nullptr;    // rows x n_cols, column-major; Q^T, or Householder vectors below R
  double* tau = nullptr;  // n_cols
  double* P = nullptr;    // n_cols x rows least-squares operator (row nu contiguous)
  double rdiag_min = 0.0, rdiag_max = 0.0;
  int lsq_method = 0;  // dpm_lsq_method of the last factorisation
  // least squares of the coupled BEPs: rcond 0 plain, > 0 truncated minimum norm; the numerical
  // rank and smallest kept singular value ratio of the last factorisation
  double rcond = 0.0;
  int rank = 0;
  double smin_ratio = 0.0;
  int kind = 1;                       // 1: Z inside Omega; 2: Z meets Gamma
  int c_off[2] = {0, 0};              // first coefficient of each subdomain's densities
  int m_rows[2] = {0, 0};             // reduced-BEP rows of each subdomain
  int32_t* row_idx[2] = {nullptr, nullptr};  // linear node index of each row (Case 2: owned)
  uint8_t* parts[2] = {nullptr, nullptr};    // Case 2: part bits of each gamma node
  int32_t* row_code = nullptr;               // Case 2: gamma_in position | part << 30 per row
  double origin[2][3] = {{0, 0, 0}, {0, 0, 0}};  // added to the node coordinates of each mesh
  // Omega_2's share of a step runs on a second stream of the handle, forked from and joined to
  // the caller's stream by events, so that the two meshes' solves overlap
  hipStream_t side = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace dpm {

dpm_status gamma_points_impl(const dpm_grid& g, const uint8_t* m_plus, int32_t* n_gamma,
                             int32_t* n_gamma_in, int32_t* idx, uint8_t* is_in, hipStream_t s);
dpm_status workspace_size_impl(const dpm_grid& g, int nrhs, const dpm_opts& o, size_t* bytes);

namespace {

constexpr int kB = 256;

unsigned blocks_for(long long n) {
  long long b = (n + kB - 1) / kB;
  return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

// M+ of Omega_1 (shell == 0: |x - c|^2 < r_in2) or of Omega_2 (shell == 1: r_in2 < |x - c|^2 <
// r_out2); nodes exactly on Z belong to neither.
__global__ void k_dd_classify(int n, double h, double x0, double cx, double cy, double cz,
                              double r_in2, double r_out2, int shell, uint8_t* __restrict__ m) {
  const long long vol = (long long)n * n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % n);
    const int iy = (int)((i / n) % n);
    const int iz = (int)(i / ((long long)n * n));
    const double px = x0 + h * ix - cx, py = x0 + h * iy - cy, pz = x0 + h * iz - cz;
    const double r2 = px * px + py * py + pz * pz;
    m[i] = (shell ? (r2 < r_out2 && r2 > r_in2) : (r2 < r_in2)) ? 1 : 0;
  }
}

// Densities of one subdomain's gamma list (rows contiguous, n_gamma entries each).  Omega_2
// (shell): rows [0, G) the Gamma part, G = (beta + 1)(m_gamma + 1), nonzero at nodes with
// |x - c| > r_split; then the Z part, 3 (m_z + 1) rows, nonzero at the other nodes.  Omega_1: the
// Z part only, at every node.  P_nu(cos theta) by the three-term recurrence, theta the polar
// angle of the node about c.
__global__ void k_dd_basis(int n, double h, double x0, double cx, double cy, double cz, int ng,
                           const int32_t* __restrict__ idx, int shell, double r_gamma,
                           int m_gamma, int beta, double r_z, int m_z, double r_split,
                           double* __restrict__ basis) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const long long li = idx[i];
  const int ix = (int)(li % n);
  const int iy = (int)((li / n) % n);
  const int iz = (int)(li / ((long long)n * n));
  const double px = x0 + h * ix - cx, py = x0 + h * iy - cy, pz = x0 + h * iz - cz;
  const double r = sqrt(px * px + py * py + pz * pz);
  const double x = cos(atan2(sqrt(px * px + py * py), pz));
  const bool on_g = shell && r > r_split;
  const long long ngl = ng;
  int row = 0;
  if (shell) {
    const int nz = m_gamma + 1;
    const double dg = r - r_gamma, hd2 = 0.5 * dg * dg;
    double pm1 = 0.0, p = 1.0;
    for (int nu = 0; nu <= m_gamma; ++nu) {
      basis[(row + nu) * ngl + i] = on_g ? p : 0.0;
      if (beta) basis[(row + nz + nu) * ngl + i] = on_g ? hd2 * p : 0.0;
      const double pn = ((2.0 * nu + 1.0) * x * p - nu * pm1) / (nu + 1.0);
      pm1 = p;
      p = pn;
    }
    row += (beta + 1) * nz;
  }
  const int nz = m_z + 1;
  const double dz = r - r_z, hd2 = 0.5 * dz * dz;
  double pm1 = 0.0, p = 1.0;
  for (int nu = 0; nu <= m_z; ++nu) {
    basis[(row + nu) * ngl + i] = on_g ? 0.0 : p;
    basis[(row + nz + nu) * ngl + i] = on_g ? 0.0 : dz * p;
    basis[(row + 2 * nz + nu) * ngl + i] = on_g ? 0.0 : hd2 * p;
    const double pn = ((2.0 * nu + 1.0) * x * p - nu * pm1) / (nu + 1.0);
    pm1 = p;
    p = pn;
  }
}

// The stacked matrix: rows [0, m0) = [0 | A_1] (Omega_1 carries only the Z columns), rows
// [m0, m0 + m1) = A_2; all column-major.
__global__ void k_dd_stack(const double* __restrict__ A0, int m0, const double* __restrict__ A1,
                           int m1, int ng_cols, int n_cols, double* __restrict__ A) {
  const long long M = (long long)m0 + m1, tot = M * n_cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e / M);
    const int i = (int)(e - (long long)j * M);
    double v;
    if (i < m0)
      v = j >= ng_cols ? A0[(long long)(j - ng_cols) * m0 + i] : 0.0;
    else
      v = A1[(long long)j * m1 + (i - m0)];
    A[e] = v;
  }
}

// g[r] = [X_1[r] at Omega_1's rows ; X_2[r] at Omega_2's rows] for the two species r =
// blockIdx.y (the rows are the reduced-BEP equations: gamma_in nodes, twice at wedge nodes)
__global__ void k_dd_gather(const double* __restrict__ X0, long long v0,
                            const int32_t* __restrict__ idx0, int m0,
                            const double* __restrict__ X1, long long v1,
                            const int32_t* __restrict__ idx1, int m1, double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int M = m0 + m1;
  if (i >= M) return;
  g[(long long)r * M + i] = i < m0 ? X0[r * v0 + idx0[i]] : X1[r * v1 + idx1[i - m0]];
}

// amp exp(-rate |x - c0|^2) at the nodes of N+, zero elsewhere
__global__ void k_dd_gauss(const uint8_t* __restrict__ np, int n, double h, double x0, double ox,
                           double oy, double oz, double amp, double rate, double cx, double cy,
                           double cz, double* __restrict__ out) {
  const long long vol = (long long)n * n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % n);
    const int iy = (int)((i / n) % n);
    const int iz = (int)(i / ((long long)n * n));
    const double px = x0 + h * ix + ox - cx, py = x0 + h * iy + oy - cy, pz = x0 + h * iz + oz - cz;
    out[i] = np[i] ? amp * exp(-rate * (px * px + py * py + pz * pz)) : 0.0;
  }
}

// ---- Case 2: Z, the sphere |x - q| = r_z about q = (0, 0, q_z), meets Gamma = {|x| = r_g} ----

struct Case2Geo {
  double r_g2;            // r_gamma^2
  double qz, rz, rz2;
  double ox, oy, oz;      // origin of the mesh
  int l;                  // subdomain: 0 the cap |x - q| < r_z, 1 the rest
};

__device__ __forceinline__ bool c2_ball(const Case2Geo& G, double X, double Y, double Z) {
  return X * X + Y * Y + Z * Z < G.r_g2;
}
__device__ __forceinline__ bool c2_zset(const Case2Geo& G, double X, double Y, double Z) {
  const double q2 = X * X + Y * Y + (Z - G.qz) * (Z - G.qz);
  return G.l == 0 ? q2 < G.rz2 : q2 > G.rz2;
}

// M+ of subdomain l: inside Gamma and on its side of Z (nodes exactly on Z in neither)
__global__ void k_dd2_classify(int n, double h, double x0, Case2Geo G, uint8_t* __restrict__ m) {
  const long long vol = (long long)n * n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % n);
    const int iy = (int)((i / n) % n);
    const int iz = (int)(i / ((long long)n * n));
    const double X = x0 + h * ix + G.ox, Y = x0 + h * iy + G.oy, Z = x0 + h * iz + G.oz;
    m[i] = (c2_ball(G, X, Y, Z) && c2_zset(G, X, Y, Z)) ? 1 : 0;
  }
}

// Whether node (ix, iy, iz) lies on the discrete grid boundary of the set given by the predicate
// (a node of the set with a neighbour in the cube outside it, or the converse)
template <bool ZSET>
__device__ bool c2_on_boundary(const Case2Geo& G, int n, double h, double x0, int ix, int iy,
                               int iz) {
  auto in = [&](int a, int b, int c) {
    const double X = x0 + h * a + G.ox, Y = x0 + h * b + G.oy, Z = x0 + h * c + G.oz;
    return ZSET ? c2_zset(G, X, Y, Z) : c2_ball(G, X, Y, Z);
  };
  const bool self = in(ix, iy, iz);
  const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int k = 0; k < 6; ++k) {
    const int a = ix + d[k][0], b = iy + d[k][1], c = iz + d[k][2];
    if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n) continue;
    if (in(a, b, c) != self) return true;
  }
  return false;
}

// Parts and effective densities of subdomain l's gamma nodes.  part bit 0: gamma_l (on the
// discrete boundary of the ball and the polar angle theta of the projection onto Gamma in the
// subdomain's window), bit 1: zeta_l (on the discrete boundary of the Z side and the angle psi of
// the projection onto Z, measured at q from the direction towards the origin, at most
// psi* + eps_z).  Rows of basis: Gamma part P_nu(cos theta), beta (d_G^2/2) P_nu, then Z part
// P_nu(cos psi), d_Z P_nu, (d_Z^2/2) P_nu, each scaled by 1/(number of parts) where the node is
// in that part, zero where it is not.  *uncovered counts nodes in no part.
__global__ void k_dd2_basis(int n, double h, double x0, Case2Geo G, int ng,
                            const int32_t* __restrict__ idx, double r_g, int m_gamma, int beta,
                            int m_z, double theta_win, double psi_win,
                            double* __restrict__ basis, uint8_t* __restrict__ part,
                            int* __restrict__ uncovered) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const long long li = idx[i];
  const int ix = (int)(li % n);
  const int iy = (int)((li / n) % n);
  const int iz = (int)(li / ((long long)n * n));
  const double X = x0 + h * ix + G.ox, Y = x0 + h * iy + G.oy, Z = x0 + h * iz + G.oz;
  const double rho = sqrt(X * X + Y * Y);
  const double rr = sqrt(X * X + Y * Y + Z * Z);
  const double rq = sqrt(X * X + Y * Y + (Z - G.qz) * (Z - G.qz));
  const double theta = atan2(rho, Z), psi = atan2(rho, G.qz - Z);
  const bool win_g = G.l == 0 ? theta <= theta_win : theta >= theta_win;
  const bool in_g = win_g && c2_on_boundary<false>(G, n, h, x0, ix, iy, iz);
  const bool in_z = psi <= psi_win && c2_on_boundary<true>(G, n, h, x0, ix, iy, iz);
  const int k = (int)in_g + (int)in_z;
  part[i] = (uint8_t)((in_g ? 1 : 0) | (in_z ? 2 : 0));
  if (k == 0) atomicAdd(uncovered, 1);
  const double w = k == 2 ? 0.5 : 1.0;
  const double wg = in_g ? w : 0.0, wz = in_z ? w : 0.0;
  const long long ngl = ng;
  {
    const int nz = m_gamma + 1;
    const double x = cos(theta);
    const double dg = rr - r_g, hd2 = 0.5 * dg * dg;
    double pm1 = 0.0, p = 1.0;
    for (int nu = 0; nu <= m_gamma; ++nu) {
      basis[nu * ngl + i] = p * wg;
      if (beta) basis[(nz + nu) * ngl + i] = hd2 * p * wg;
      const double pn = ((2.0 * nu + 1.0) * x * p - nu * pm1) / (nu + 1.0);
      pm1 = p;
      p = pn;
    }
  }
  {
    const int row = (beta + 1) * (m_gamma + 1);
    const int nz = m_z + 1;
    const double x = cos(psi);
    const double dz = rq - G.rz, hd2 = 0.5 * dz * dz;
    double pm1 = 0.0, p = 1.0;
    for (int nu = 0; nu <= m_z; ++nu) {
      basis[(row + nu) * ngl + i] = p * wz;
      basis[(row + nz + nu) * ngl + i] = dz * p * wz;
      basis[(row + 2 * nz + nu) * ngl + i] = hd2 * p * wz;
      const double pn = ((2.0 * nu + 1.0) * x * p - nu * pm1) / (nu + 1.0);
      pm1 = p;
      p = pn;
    }
  }
}

// Rows [r0, r0 + nr) of the stacked matrix from subdomain l's columns A_l = B_eff|gamma_in -
// Tr P B_eff (n_in x n_cols, column-major) and effective densities B_eff (n_cols x n_gamma): a
// row of part Gamma (Z) at gamma_in node i (gamma position j) is -Tr_i P B_eff plus the node's
// own, unscaled Gamma (Z) densities.  row_node: i | part << 30.
__global__ void k_dd2_stack(const double* __restrict__ Al, int n_in, const double* __restrict__ B,
                            int ng, const int32_t* __restrict__ pos_in,
                            const uint8_t* __restrict__ part, const int32_t* __restrict__ row_node,
                            int nr, int ng_cols, int n_cols, int r0, int M,
                            double* __restrict__ A) {
  const long long tot = (long long)nr * n_cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int nu = (int)(e / nr);
    const int r = (int)(e - (long long)nu * nr);
    const int code = row_node[r];
    const int i = code & 0x3fffffff, zpart = code >> 30;
    const int j = pos_in[i];
    const int k = (part[j] & 1) + ((part[j] >> 1) & 1);
    const bool own = zpart ? nu >= ng_cols : nu < ng_cols;
    const double a = Al[(long long)nu * n_in + i];
    double v;
    if (own && k == 1)
      v = a;  // the effective density is the node's own: A_l's row as it is
    else {
      const double b = B[(long long)nu * ng + j];
      v = a - b + (own ? k * b : 0.0);
    }
    A[(long long)nu * M + r0 + r] = v;
  }
}

struct DDLayout {
  size_t b2[2], X[2], ug[2], g, C, solve_ws[2], total;
};

DDLayout dd_layout(const dpm_dd* d, size_t solve_ws) {
  DDLayout L;
  size_t o = 0;
  for (int l = 0; l < 2; ++l) {
    const dpm_grid& g = d->sub[l]->grid;
    const size_t V = (size_t)g.n * g.n * g.n * sizeof(double);
    L.b2[l] = o; o = align_up(o + 2 * V, 256);
    L.X[l] = o; o = align_up(o + 2 * V, 256);
    L.ug[l] = o; o = align_up(o + 2 * sizeof(double) * d->sub[l]->n_gamma, 256);
  }
  L.g = o; o = align_up(o + 2 * sizeof(double) * d->rows, 256);
  L.C = o; o = align_up(o + 2 * sizeof(double) * d->n_cols, 256);
  for (int l = 0; l < 2; ++l) { L.solve_ws[l] = o; o = align_up(o + solve_ws, 256); }
  L.total = o;
  return L;
}

dpm_status dd_solve_ws(const dpm_dd* d, const dpm_opts& o, size_t* bytes) {
  size_t mx = 0;
  dpm_opts so = o;
  so.rhs_chunk = 2;  // both species in one launch: the size never depends on tuning
  for (int l = 0; l < 2; ++l) {
    size_t w = 0;
    DPM_TRY(workspace_size_impl(d->sub[l]->grid, 2, so, &w));
    if (w > mx) mx = w;
  }
  *bytes = mx;
  return DPM_OK;
}

}  // namespace

void dd_destroy(dpm_dd* d) {
  if (!d) return;
  if (d->kind == 2) {
    for (int32_t* p : d->row_idx) (void)hipFree(p);
    for (uint8_t* p : d->parts) (void)hipFree(p);
    (void)hipFree(d->row_code);
  }
  for (hipEvent_t e : d->ev)
    if (e) (void)hipEventDestroy(e);
  if (d->side) (void)hipStreamDestroy(d->side);
  destroy_bep(d->sub[0]);
  destroy_bep(d->sub[1]);
  (void)hipFree(d->A);
  (void)hipFree(d->tau);
  (void)hipFree(d->P);
  delete d;
}

// The stacked matrix from the subdomains' columns (Case 1: [[0, A_1], [A_2]]; Case 2: the rows
// of both parts), A_out (nullable) a copy before factorisation, then QR, rank test and P.
dpm_status dd_stack_factor(dpm_dd* d, hipStream_t s, double* A_out, void* scratch, size_t bytes,
                           double* rd2) {
  const size_t na = (size_t)d->rows * d->n_cols;
  if (d->kind == 1) {
    hipLaunchKernelGGL(k_dd_stack, dim3(blocks_for((long long)na)), dim3(kB), 0, s, d->sub[0]->A,
                       d->sub[0]->n_in, d->sub[1]->A, d->sub[1]->n_in, d->n_gamma_cols, d->n_cols,
                       d->A);
  } else {
    for (int l = 0; l < 2; ++l) {
      const dpm_bep* b = d->sub[l];
      const int r0 = l == 0 ? 0 : d->m_rows[0];
      hipLaunchKernelGGL(k_dd2_stack, dim3(blocks_for((long long)d->m_rows[l] * d->n_cols)),
                         dim3(kB), 0, s, b->A, b->n_in, b->basis, b->n_gamma, b->pos_in,
                         d->parts[l], d->row_code + r0, d->m_rows[l], d->n_gamma_cols, d->n_cols,
                         r0, d->rows, d->A);
    }
  }
  DPM_TRY_HIP(hipGetLastError());
  if (A_out) DPM_TRY_HIP(hipMemcpyAsync(A_out, d->A, sizeof(double) * na, hipMemcpyDeviceToDevice, s));
  return lsq_factor(d->A, d->rows, d->n_cols, d->tau, d->P, s, scratch, bytes, rd2, d->rcond,
                    &d->lsq_method);
}

// Result of a factorisation read back from rd[0..3]: (min, max) |R_ii|, and with truncation the
// numerical rank and smallest kept singular value ratio.  Plain least squares needs full column
// rank (rank_check); the truncated one has no such condition.
dpm_status dd_rank_result(dpm_dd* d, const double* rd) {
  d->rdiag_min = rd[0];
  d->rdiag_max = rd[1];
  if (d->rcond > 0.0) {
    d->rank = (int)rd[2];
    d->smin_ratio = rd[3];
    if (!(d->rank > 0)) {
      set_error("truncated least squares kept no singular value (rank %d)", d->rank);
      return DPM_ERANK;
    }
    return DPM_OK;
  }
  d->rank = d->n_cols;
  d->smin_ratio = 0.0;
  return rank_check(rd[0], rd[1]);
}

// Scratch of a rebuild: the subdomains' column builds run one after the other, then the stacked
// factorisation, all on one stream, so they share it.
size_t dd_rebuild_scratch_bytes(const dpm_dd* d) {
  size_t mx = factor_scratch_bytes(d->rows, d->n_cols);
  for (int l = 0; l < 2; ++l) {
    const size_t c = columns_scratch_bytes(d->sub[l]);
    if (c > mx) mx = c;
  }
  return mx;
}

// Both subdomains' columns, the stacked matrix, its QR and P (enqueue only; rd2 as lsq_factor).
dpm_status dd_factor_enqueue(dpm_dd* d, hipStream_t s, double* A_out, void* scratch, size_t bytes,
                             double* rd2) {
  for (int l = 0; l < 2; ++l) DPM_TRY(bep_columns(d->sub[l], s, scratch, bytes));
  return dd_stack_factor(d, s, A_out, scratch, bytes, rd2);
}

// The same with one synchronisation for the rank test (rd2 at the end of the scratch).
dpm_status dd_factor(dpm_dd* d, hipStream_t s, double* A_out, void* scratch, size_t bytes) {
  if (scratch == nullptr || bytes < dd_rebuild_scratch_bytes(d) + 256) {
    set_error("decomposed-domain build: scratch too small: %zu bytes given, %zu needed", bytes,
              dd_rebuild_scratch_bytes(d) + 256);
    return DPM_EINVAL;
  }
  double* rd2 = reinterpret_cast<double*>(static_cast<char*>(scratch) + (bytes - 256) / 256 * 256);
  DPM_TRY(dd_factor_enqueue(d, s, A_out, scratch, bytes - 256, rd2));
  double h4[4] = {0.0, 0.0, 0.0, 0.0};
  DPM_TRY_HIP(hipMemcpyAsync(h4, rd2, sizeof(h4), hipMemcpyDeviceToHost, s));
  DPM_TRY_HIP(hipStreamSynchronize(s));
  return dd_rank_result(d, h4);
}

// The build's stacking and factorisation (Step 2 creates the handle; the subdomains' columns are
// already built): scratch allocated, used and freed here, one synchronisation, rank test.
dpm_status dd_stack_factor_alloc(dpm_dd* d, hipStream_t s, double* A_out) {
  const size_t fb = align_up(factor_scratch_bytes(d->rows, d->n_cols), 256);
  void* scratch = nullptr;
  if (hipMalloc(&scratch, fb + 256) != hipSuccess) {
    set_error("decomposed-domain build: device allocation of %zu scratch bytes failed", fb + 256);
    return DPM_ENOMEM;
  }
  double* rd2 = reinterpret_cast<double*>(static_cast<char*>(scratch) + fb);
  double h2[4] = {0.0, 0.0, 0.0, 0.0};
  dpm_status st = dd_stack_factor(d, s, A_out, scratch, fb, rd2);
  hipError_t e = hipSuccess;
  if (st == DPM_OK) e = hipMemcpyAsync(h2, rd2, sizeof(h2), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  (void)hipFree(scratch);
  if (st == DPM_OK && e != hipSuccess) {
    set_error("decomposed-domain build: %s", hipGetErrorString(e));
    st = DPM_EHIP;
  }
  if (st != DPM_OK) return st;
  return dd_rank_result(d, h2);
}

dpm_status dd_build_impl(const dpm_dd_params& prm, const dpm_opts& o, hipStream_t s,
                         dpm_dd** out, double* A_out) {
  dpm_dd* d = new dpm_dd();
  d->prm = prm;
  d->n_gamma_cols = (prm.beta + 1) * (prm.m_gamma + 1);
  d->n_z_cols = 3 * (prm.m_z + 1);
  d->n_cols = d->n_gamma_cols + d->n_z_cols;
  auto fail = [&](dpm_status st) {
    dd_destroy(d);
    return st;
  };
  if (hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking) != hipSuccess) {
    set_error("dpm_dd_build: stream creation failed");
    return fail(DPM_EHIP);
  }
  for (hipEvent_t& e : d->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      set_error("dpm_dd_build: event creation failed");
      return fail(DPM_EHIP);
    }
  const double* c = prm.center;
  for (int l = 0; l < 2; ++l) {
    const dpm_grid& g = l == 0 ? prm.grid1 : prm.grid2;
    const long long vsz = (long long)g.n * g.n * g.n;
    uint8_t* m = nullptr;
    int32_t* idx = nullptr;
    uint8_t* is_in = nullptr;
    double* basis = nullptr;
    auto release = [&]() {
      (void)hipFree(m); (void)hipFree(idx); (void)hipFree(is_in); (void)hipFree(basis);
    };
    if (hipMalloc(&m, vsz) != hipSuccess) {
      set_error("dpm_dd_build: device allocation failed");
      return fail(DPM_ENOMEM);
    }
    hipLaunchKernelGGL(k_dd_classify, dim3(blocks_for(vsz)), dim3(kB), 0, s, g.n, g.h, g.x0, c[0],
                       c[1], c[2], prm.r_z * prm.r_z, prm.r_gamma * prm.r_gamma, l, m);
    int32_t ng = 0, nin = 0;
    dpm_status st = gamma_points_impl(g, m, &ng, &nin, nullptr, nullptr, s);
    if (st != DPM_OK) { release(); return fail(st); }
    const int nb = l == 0 ? d->n_z_cols : d->n_cols;
    if (hipMalloc(&idx, sizeof(int32_t) * ng) != hipSuccess || hipMalloc(&is_in, ng) != hipSuccess ||
        hipMalloc(&basis, sizeof(double) * (size_t)nb * ng) != hipSuccess) {
      release();
      set_error("dpm_dd_build: device allocation failed");
      return fail(DPM_ENOMEM);
    }
    st = gamma_points_impl(g, m, &ng, &nin, idx, is_in, s);
    if (st != DPM_OK) { release(); return fail(st); }
    hipLaunchKernelGGL(k_dd_basis, dim3((ng + 127) / 128), dim3(128), 0, s, g.n, g.h, g.x0, c[0],
                       c[1], c[2], ng, idx, l, prm.r_gamma, prm.m_gamma, prm.beta, prm.r_z,
                       prm.m_z, prm.r_split, basis);
    if (hipGetLastError() != hipSuccess) {
      release();
      set_error("dpm_dd_build: kernel launch failed");
      return fail(DPM_EHIP);
    }
    // point sets, densities and the unfactored columns A_l of this subdomain
    st = build_bep_impl(g, m, nb, basis, o, s, &d->sub[l], nullptr, false);
    (void)hipStreamSynchronize(s);
    release();
    if (st != DPM_OK) return fail(st);
  }
  const int m0 = d->sub[0]->n_in, m1 = d->sub[1]->n_in;
  d->rows = m0 + m1;
  d->kind = 1;
  d->c_off[0] = d->n_gamma_cols;
  for (int l = 0; l < 2; ++l) {
    d->m_rows[l] = d->sub[l]->n_in;
    d->row_idx[l] = d->sub[l]->idx_in;  // every gamma_in node once, owned by the subdomain
  }
  if (d->n_cols > d->rows) {
    set_error("dpm_dd_build: %d columns exceed the %d rows of the coupled BEP", d->n_cols, d->rows);
    return fail(DPM_ERANK);
  }
  const size_t na = (size_t)d->rows * d->n_cols;
  if (hipMalloc(&d->A, sizeof(double) * na) != hipSuccess ||
      hipMalloc(&d->tau, sizeof(double) * d->n_cols) != hipSuccess ||
      hipMalloc(&d->P, sizeof(double) * na) != hipSuccess) {
    set_error("dpm_dd_build: device allocation failed");
    return fail(DPM_ENOMEM);
  }
  {
    const dpm_status st = dd_stack_factor_alloc(d, s, A_out);
    if (st != DPM_OK) return fail(st);
  }
  *out = d;
  return DPM_OK;
}

dpm_status dd2_build_impl(const dpm_dd2_params& prm, const dpm_opts& o, hipStream_t s,
                          dpm_dd** out, double* A_out) {
  dpm_dd* d = new dpm_dd();
  d->kind = 2;
  d->rcond = prm.rcond;
  d->n_gamma_cols = (prm.beta + 1) * (prm.m_gamma + 1);
  d->n_z_cols = 3 * (prm.m_z + 1);
  d->n_cols = d->n_gamma_cols + d->n_z_cols;
  d->prm.grid1 = prm.grid1;
  d->prm.grid2 = prm.grid2;
  auto fail = [&](dpm_status st) {
    dd_destroy(d);
    return st;
  };
  if (hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking) != hipSuccess) {
    set_error("dpm_dd2_build: stream creation failed");
    return fail(DPM_EHIP);
  }
  for (hipEvent_t& e : d->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      set_error("dpm_dd2_build: event creation failed");
      return fail(DPM_EHIP);
    }
  // the circle where Z meets Gamma
  const double rg = prm.r_gamma, qz = prm.q_z, rz = prm.r_z;
  const double z_star = (rg * rg + qz * qz - rz * rz) / (2.0 * qz);
  const double theta_star = std::acos(z_star / rg), psi_star = std::acos((qz - z_star) / rz);
  uint8_t** parts = d->parts;  // kept for rebuilds; freed with the handle
  for (int l = 0; l < 2; ++l) {
    const dpm_grid& g = l == 0 ? prm.grid1 : prm.grid2;
    const double* org = l == 0 ? prm.origin1 : prm.origin2;
    for (int a = 0; a < 3; ++a) d->origin[l][a] = org[a];
    Case2Geo G{rg * rg, qz, rz, rz * rz, org[0], org[1], org[2], l};
    const long long vsz = (long long)g.n * g.n * g.n;
    uint8_t* m = nullptr;
    int32_t* idx = nullptr;
    uint8_t* is_in = nullptr;
    double* basis = nullptr;
    int* unc = nullptr;
    auto release = [&]() {
      (void)hipFree(m); (void)hipFree(idx); (void)hipFree(is_in); (void)hipFree(basis);
      (void)hipFree(unc);
    };
    if (hipMalloc(&m, vsz) != hipSuccess || hipMalloc(&unc, sizeof(int)) != hipSuccess) {
      release();
      set_error("dpm_dd2_build: device allocation failed");
      return fail(DPM_ENOMEM);
    }
    hipLaunchKernelGGL(k_dd2_classify, dim3(blocks_for(vsz)), dim3(kB), 0, s, g.n, g.h, g.x0, G, m);
    int32_t ng = 0, nin = 0;
    dpm_status st = gamma_points_impl(g, m, &ng, &nin, nullptr, nullptr, s);
    if (st != DPM_OK) { release(); return fail(st); }
    const int nb = d->n_cols;
    if (hipMalloc(&idx, sizeof(int32_t) * ng) != hipSuccess || hipMalloc(&is_in, ng) != hipSuccess ||
        hipMalloc(&basis, sizeof(double) * (size_t)nb * ng) != hipSuccess ||
        hipMalloc(&parts[l], ng) != hipSuccess) {
      release();
      set_error("dpm_dd2_build: device allocation failed");
      return fail(DPM_ENOMEM);
    }
    st = gamma_points_impl(g, m, &ng, &nin, idx, is_in, s);
    if (st != DPM_OK) { release(); return fail(st); }
    const double eps = prm.eps_layers * g.h;
    const double theta_win = l == 0 ? theta_star + eps / rg : theta_star - eps / rg;
    const double psi_win = psi_star + eps / rz;
    int uncovered = 0;
    hipError_t e = hipMemsetAsync(unc, 0, sizeof(int), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_dd2_basis, dim3((ng + 127) / 128), dim3(128), 0, s, g.n, g.h, g.x0, G,
                         ng, idx, rg, prm.m_gamma, prm.beta, prm.m_z, theta_win, psi_win, basis,
                         parts[l], unc);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&uncovered, unc, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      release();
      set_error("dpm_dd2_build: %s", hipGetErrorString(e));
      return fail(DPM_EHIP);
    }
    if (uncovered > 0) {
      release();
      set_error("dpm_dd2_build: %d nodes of subdomain %d's discrete boundary lie in neither gamma_l "
                "nor zeta_l: raise eps_layers", uncovered, l + 1);
      return fail(DPM_EGEOM);
    }
    st = build_bep_impl(g, m, nb, basis, o, s, &d->sub[l], nullptr, false);
    (void)hipStreamSynchronize(s);
    release();
    if (st != DPM_OK) return fail(st);
  }
  // rows: gamma_in nodes in ascending index, a Gamma row and then a Z row at wedge nodes
  std::vector<int32_t> rn[2];
  for (int l = 0; l < 2; ++l) {
    const dpm_bep* b = d->sub[l];
    std::vector<uint8_t> pt(b->n_gamma);
    std::vector<int32_t> pos(b->n_in), idx_in(b->n_in);
    hipError_t e = hipMemcpy(pt.data(), parts[l], b->n_gamma, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(pos.data(), b->pos_in, sizeof(int32_t) * b->n_in, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(idx_in.data(), b->idx_in, sizeof(int32_t) * b->n_in, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_error("dpm_dd2_build: %s", hipGetErrorString(e));
      return fail(DPM_EHIP);
    }
    std::vector<int32_t> ridx;
    for (int i = 0; i < b->n_in; ++i) {
      const uint8_t p = pt[pos[i]];
      if (p & 1) { rn[l].push_back(i); ridx.push_back(idx_in[i]); }
      if (p & 2) { rn[l].push_back(i | (1 << 30)); ridx.push_back(idx_in[i]); }
    }
    d->m_rows[l] = (int)ridx.size();
    if (hipMalloc(&d->row_idx[l], sizeof(int32_t) * (ridx.size() + 1)) != hipSuccess ||
        hipMemcpy(d->row_idx[l], ridx.data(), sizeof(int32_t) * ridx.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("dpm_dd2_build: device allocation or copy failed");
      return fail(DPM_ENOMEM);
    }
  }
  d->rows = d->m_rows[0] + d->m_rows[1];
  if (d->n_cols > d->rows) {
    set_error("dpm_dd2_build: %d columns exceed the %d rows of the coupled BEP", d->n_cols, d->rows);
    return fail(DPM_ERANK);
  }
  const size_t na = (size_t)d->rows * d->n_cols;
  if (hipMalloc(&d->A, sizeof(double) * na) != hipSuccess ||
      hipMalloc(&d->tau, sizeof(double) * d->n_cols) != hipSuccess ||
      hipMalloc(&d->P, sizeof(double) * na) != hipSuccess ||
      hipMalloc(&d->row_code, sizeof(int32_t) * (size_t)d->rows) != hipSuccess) {
    set_error("dpm_dd2_build: device allocation failed");
    return fail(DPM_ENOMEM);
  }
  int32_t* drn = d->row_code;
  hipError_t e = hipMemcpy(drn, rn[0].data(), sizeof(int32_t) * rn[0].size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(drn + rn[0].size(), rn[1].data(), sizeof(int32_t) * rn[1].size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("dpm_dd2_build: %s", hipGetErrorString(e));
    return fail(DPM_EHIP);
  }
  {
    const dpm_status st = dd_stack_factor_alloc(d, s, A_out);
    if (st != DPM_OK) return fail(st);
  }
  *out = d;
  return DPM_OK;
}

void dd_set_sigma(dpm_dd* d, double sigma) {
  d->prm.grid1.sigma = sigma;
  d->prm.grid2.sigma = sigma;
  for (int l = 0; l < 2; ++l) d->sub[l]->grid.sigma = sigma;
}

size_t dd_rebuild_workspace_bytes(const dpm_dd* d) { return dd_rebuild_scratch_bytes(d) + 256; }

dpm_status dd_rebuild_impl(dpm_dd* d, double sigma, hipStream_t s, void* scratch, size_t bytes) {
  if (scratch == nullptr || bytes < dd_rebuild_workspace_bytes(d)) {
    set_error("dpm_dd_rebuild: workspace too small: %zu bytes given, %zu needed", bytes,
              dd_rebuild_workspace_bytes(d));
    return DPM_EINVAL;
  }
  dd_set_sigma(d, sigma);
  return dd_factor(d, s, nullptr, scratch, bytes);
}

double dd_sigma(const dpm_dd* d) { return d->prm.grid1.sigma; }
const dpm_bep* dd_sub(const dpm_dd* d, int l) { return d->sub[l]; }
const double* dd_origin(const dpm_dd* d, int l) { return d->origin[l]; }

int dd_lsq_method(const dpm_dd* d) { return d->lsq_method; }

dpm_status dd_lsq_info_impl(const dpm_dd* d, double* rcond, int32_t* rank, double* smin_ratio) {
  if (rcond) *rcond = d->rcond;
  if (rank) *rank = d->rank;
  if (smin_ratio) *smin_ratio = d->smin_ratio;
  return DPM_OK;
}

dpm_status dd_info_impl(const dpm_dd* d, int32_t n_gamma[2], int32_t n_in[2], int32_t n_rows[2],
                        int32_t* n_cols, double* rmin, double* rmax) {
  for (int l = 0; l < 2; ++l) {
    if (n_gamma) n_gamma[l] = d->sub[l]->n_gamma;
    if (n_in) n_in[l] = d->sub[l]->n_in;
    if (n_rows) n_rows[l] = d->m_rows[l];
  }
  if (n_cols) *n_cols = d->n_cols;
  if (rmin) *rmin = d->rdiag_min;
  if (rmax) *rmax = d->rdiag_max;
  return DPM_OK;
}

dpm_status dd_step_workspace_impl(const dpm_dd* d, const dpm_opts& o, size_t* bytes) {
  size_t sw = 0;
  DPM_TRY(dd_solve_ws(d, o, &sw));
  *bytes = dd_layout(d, sw).total;
  return DPM_OK;
}

dpm_status dd_run_workspace_impl(const dpm_dd* d, const dpm_opts& o, size_t* bytes) {
  size_t need = 0;
  DPM_TRY(dd_step_workspace_impl(d, o, &need));
  *bytes = align_up(need, 256) + 256 + align_up(dd_rebuild_scratch_bytes(d), 256);
  return DPM_OK;
}

dpm_status dd_step_impl(const dpm_dd* d, double dt, double chi, const double* const in[4],
                        double* const out[4], const dpm_opts& o, hipStream_t s) {
  size_t sw = 0;
  DPM_TRY(dd_solve_ws(d, o, &sw));
  const DDLayout L = dd_layout(d, sw);
  if (o.workspace == nullptr || o.workspace_bytes < L.total) {
    set_error("dpm_dd_step: workspace too small: %zu bytes given, %zu needed", o.workspace_bytes,
              L.total);
    return DPM_EINVAL;
  }
  char* ws = static_cast<char*>(o.workspace);
  dpm_opts so[2] = {o, o};
  double* b2[2];
  double* X[2];
  double* ug[2];
  for (int l = 0; l < 2; ++l) {
    so[l].rhs_chunk = 2;
    so[l].workspace = ws + L.solve_ws[l];
    so[l].workspace_bytes = sw;
    b2[l] = reinterpret_cast<double*>(ws + L.b2[l]);
    X[l] = reinterpret_cast<double*>(ws + L.X[l]);
    ug[l] = reinterpret_cast<double*>(ws + L.ug[l]);
  }
  double* g = reinterpret_cast<double*>(ws + L.g);
  double* C = reinterpret_cast<double*>(ws + L.C);
  hipStream_t st[2] = {s, d->side};
  // Step 4a on both meshes (Omega_2 on the side stream): forcing and particular solutions
  DPM_TRY_HIP(hipEventRecord(d->ev[0], s));
  DPM_TRY_HIP(hipStreamWaitEvent(d->side, d->ev[0], 0));
  for (int l = 0; l < 2; ++l) {
    launch_pks_rhs(d->sub[l], in[2 * l], in[2 * l + 1], dt, chi, b2[l], st[l]);
    DPM_TRY_HIP(hipGetLastError());
    DPM_TRY(aux_solve_impl(d->sub[l]->grid, 2, b2[l], X[l], so[l], st[l], nullptr));
  }
  DPM_TRY_HIP(hipEventRecord(d->ev[1], d->side));
  DPM_TRY_HIP(hipStreamWaitEvent(s, d->ev[1], 0));
  // Step 5: the coupled least squares on the stacked traces
  const dpm_bep* s0 = d->sub[0];
  const dpm_bep* s1 = d->sub[1];
  const long long v0 = (long long)s0->grid.n * s0->grid.n * s0->grid.n;
  const long long v1 = (long long)s1->grid.n * s1->grid.n * s1->grid.n;
  hipLaunchKernelGGL(k_dd_gather, dim3((d->rows + kB - 1) / kB, 2), dim3(kB), 0, s, X[0], v0,
                     d->row_idx[0], d->m_rows[0], X[1], v1, d->row_idx[1], d->m_rows[1], g);
  lsq_apply(d->P, d->rows, d->n_cols, 2, g, C, s);
  // densities (Case 1: Omega_1 from the Z coefficients only)
  launch_density(s0, C + d->c_off[0], d->n_cols, ug[0], s);
  launch_density(s1, C + d->c_off[1], d->n_cols, ug[1], s);
  DPM_TRY_HIP(hipGetLastError());
  // Steps 6-7 per subdomain: Green's formula as one AP solve per species, restriction to N+
  DPM_TRY_HIP(hipEventRecord(d->ev[2], s));
  DPM_TRY_HIP(hipStreamWaitEvent(d->side, d->ev[2], 0));
  for (int l = 0; l < 2; ++l) {
    minus_rhs(d->sub[l], ug[l], 0, 2, b2[l], st[l]);
    DPM_TRY_HIP(hipGetLastError());
    if (restrict_fusable(d->sub[l]->grid, so[l])) {
      // the restriction to N+ in the solve's last pass
      const RestrictOut ro{d->sub[l]->n_plus, out[2 * l], out[2 * l + 1], nullptr};
      DPM_TRY(aux_solve_impl(d->sub[l]->grid, 2, b2[l], X[l], so[l], st[l], nullptr, nullptr,
                             false, 0, &ro));
    } else {
      DPM_TRY(aux_solve_impl(d->sub[l]->grid, 2, b2[l], X[l], so[l], st[l], nullptr));
      launch_restrict(d->sub[l], X[l], out[2 * l], out[2 * l + 1], st[l]);
    }
    DPM_TRY_HIP(hipGetLastError());
  }
  DPM_TRY_HIP(hipEventRecord(d->ev[3], d->side));
  DPM_TRY_HIP(hipStreamWaitEvent(s, d->ev[3], 0));
  return DPM_OK;
}

// The adaptive loop of the paper's algorithm on the decomposed domain: the CFL-type bound of
// each subdomain on its own mesh (h_l / (6 chi max|grad_h c_l|)), the smaller of the two, Step 4b
// rebuilds of both subdomains' columns and of the coupled QR when dt shrinks, Step 8 on
// max |rho| over both M+.
dpm_status dd_run_impl(dpm_dd* d, const dpm_run_params& p, double* const state[4],
                       const dpm_opts& o, hipStream_t s, dpm_run_info* info, double* dt_hist,
                       uint8_t* rebuilt_hist) {
  size_t need = 0;
  DPM_TRY(dd_step_workspace_impl(d, o, &need));
  const size_t scan_off = align_up(need, 256);
  const size_t reb_off = scan_off + 256;
  const size_t reb_bytes = align_up(dd_rebuild_scratch_bytes(d), 256);
  if (o.workspace == nullptr || o.workspace_bytes < reb_off + reb_bytes) {
    set_error("dpm_dd_run: workspace too small: %zu bytes given, %zu needed", o.workspace_bytes,
              reb_off + reb_bytes);
    return DPM_EINVAL;
  }
  // scan[0..3]: both subdomains' scanned maxima; scan[4..7]: (min, max) |R_ii|, rank and
  // smallest kept singular value ratio of the last rebuild, read back with the next scan (a
  // rebuild adds no synchronisation of its own)
  double* scan = reinterpret_cast<double*>(static_cast<char*>(o.workspace) + scan_off);
  void* rscratch = static_cast<char*>(o.workspace) + reb_off;
  dpm_run_info r{};
  r.stop = DPM_RUN_MAXSTEPS;
  double t = 0.0, dt_prev = 1.0 / d->prm.grid1.sigma;
  double rho_prev = 0.0;  // max |rho| of the previous scan (none before the first)
  const double* in[4] = {state[0], state[1], state[2], state[3]};
  bool rank_pending = false;
  for (;;) {
    double w[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool more = t < p.t_final && r.steps < p.max_steps;
    if (more)
      for (int l = 0; l < 2; ++l)
        DPM_TRY(cfl_scan_impl(d->sub[l], state[2 * l], state[2 * l + 1], scan + 2 * l, s));
    if (more || rank_pending) {
      DPM_TRY_HIP(hipMemcpyAsync(w, scan, sizeof(w), hipMemcpyDeviceToHost, s));
      DPM_TRY_HIP(hipStreamSynchronize(s));
    }
    if (rank_pending) {
      rank_pending = false;
      DPM_TRY(dd_rank_result(d, w + 4));
    }
    if (t >= p.t_final) { r.stop = DPM_RUN_TFINAL; break; }
    if (r.steps >= p.max_steps) { r.stop = DPM_RUN_MAXSTEPS; break; }
    const double v[4] = {w[0], w[1], w[2], w[3]};
    r.grad_max = std::fmax(v[0], v[2]);
    r.rho_max = std::fmax(v[1], v[3]);
    bool finite = true;
    for (double x : v) finite = finite && std::isfinite(x);
    if (!finite) {
      r.grad_max = r.rho_max = NAN;
      r.stop = DPM_RUN_NONFINITE;
      break;
    }
    if (r.rho_max > p.rho_cap) { r.stop = DPM_RUN_RHOCAP; break; }
    if (p.rho_jump_cap > 0.0 && r.steps > 0 && r.rho_max - rho_prev >= p.rho_jump_cap) {
      r.stop = DPM_RUN_RHOJUMP;
      break;
    }
    rho_prev = r.rho_max;
    double dt = dt_prev;
    for (int l = 0; l < 2; ++l)
      if (v[2 * l] > 0.0) {
        const double dt_cfl = d->sub[l]->grid.h / (6.0 * p.chi * v[2 * l]);
        if (dt_cfl < dt) dt = dt_cfl;
      }
    const bool rebuild = dt < dt_prev;
    if (rebuild) {
      dd_set_sigma(d, 1.0 / dt);
      DPM_TRY(dd_factor_enqueue(d, s, nullptr, rscratch, reb_bytes, scan + 4));
      rank_pending = true;
      ++r.rebuilds;
    }
    DPM_TRY(dd_step_impl(d, dt, p.chi, in, state, o, s));
    if (dt_hist) dt_hist[r.steps] = dt;
    if (rebuilt_hist) rebuilt_hist[r.steps] = rebuild ? 1 : 0;
    ++r.steps;
    t += dt;
    dt_prev = dt;
  }
  DPM_TRY_HIP(hipStreamSynchronize(s));
  r.t = t;
  r.dt = dt_prev;
  if (info) *info = r;
  return DPM_OK;
}

// A decomposed step on fixed buffers, captured into a HIP graph: the side stream's branch joins
// the capture through the fork and join events, so one replay runs both meshes' work.
struct DDStepper {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

dpm_status dd_stepper_create_impl(const dpm_dd* d, double dt, double chi, double* const state[4],
                                  const dpm_opts& o, void** out) {
  if (timing_enabled()) {
    set_error("dpm_dd_stepper_create: sweep timing is enabled; end it before capturing a step");
    return DPM_EINVAL;
  }
  for (int l = 0; l < 2; ++l) {
    const Plan* pl = nullptr;
    DPM_TRY(get_plan(d->sub[l]->grid.n, &pl));  // tables exist before capture
  }
  hipStream_t cs = nullptr;
  DPM_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    set_error("dpm_dd_stepper_create: hipStreamBeginCapture: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  const double* in[4] = {state[0], state[1], state[2], state[3]};
  const dpm_status st = dd_step_impl(d, dt, chi, in, state, o, cs);
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (st != DPM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error("dpm_dd_stepper_create: graph capture: %s", hipGetErrorString(e));
    return DPM_EHIP;
  }
  auto* p = new DDStepper;
  p->graph = graph;
  p->exec = exec;
  *out = p;
  return DPM_OK;
}

dpm_status dd_stepper_run_impl(void* h, int nsteps, hipStream_t s) {
  auto* p = static_cast<DDStepper*>(h);
  for (int k = 0; k < nsteps; ++k) DPM_TRY_HIP(hipGraphLaunch(p->exec, s));
  return DPM_OK;
}

void dd_stepper_destroy_impl(void* h) {
  auto* p = static_cast<DDStepper*>(h);
  if (!p) return;
  (void)hipDeviceSynchronize();  // replays still in flight finish before the graph goes
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

dpm_status dd_masks_impl(const dpm_dd* d, int l, uint8_t* m_plus, uint8_t* n_plus, hipStream_t s) {
  const dpm_bep* b = d->sub[l];
  const size_t vsz = (size_t)b->grid.n * b->grid.n * b->grid.n;
  if (m_plus) DPM_TRY_HIP(hipMemcpyAsync(m_plus, b->m_plus, vsz, hipMemcpyDeviceToDevice, s));
  if (n_plus) DPM_TRY_HIP(hipMemcpyAsync(n_plus, b->n_plus, vsz, hipMemcpyDeviceToDevice, s));
  return DPM_OK;
}

dpm_status dd_gauss_impl(const dpm_dd* d, int l, double amp, double rate, const double c0[3],
                         double* out, hipStream_t s) {
  const dpm_bep* b = d->sub[l];
  const dpm_grid& g = b->grid;
  const long long vsz = (long long)g.n * g.n * g.n;
  const double* o = d->origin[l];
  hipLaunchKernelGGL(k_dd_gauss, dim3(blocks_for(vsz)), dim3(kB), 0, s, b->n_plus, g.n, g.h, g.x0,
                     o[0], o[1], o[2], amp, rate, c0[0], c0[1], c0[2], out);
  DPM_TRY_HIP(hipGetLastError());
  return DPM_OK;
}

}  // namespace dpm
