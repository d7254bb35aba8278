/*
 * A C program that drives libdpm through its C ABI alone (no Python): one auxiliary-problem solve
 * of a sine mode checked against its closed form, the argument checks, and a short DPM time loop
 * on the unit sphere (classification, discrete boundary, densities, boundary matrix, captured
 * steps), the adaptive loop, and the adaptive loop of the domain decomposition (Case 2).  Prints
 * "ok" and returns 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "dpm.h"

#define CHECK(call)                                                                   \
  do {                                                                                \
    dpm_status st_ = (call);                                                          \
    if (st_ != DPM_OK) {                                                              \
      fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, dpm_last_error());     \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)
#define HCHECK(call)                                                                  \
  do {                                                                                \
    if ((call) != hipSuccess) {                                                       \
      fprintf(stderr, "%s failed\n", #call);                                          \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

static const double kPi = 3.14159265358979323846;

int main(void) {
  const int n = 31;
  const double h = 3.0 / (n + 1), x0 = -1.5 + h, sigma = 2.0;
  const size_t vol = (size_t)n * n * n;

  /* ---- 1. sine mode (k1, k2, k3): u = b / (sigma + lambda_k1 + lambda_k2 + lambda_k3) */
  const int k1 = 3, k2 = 17, k3 = 31;
  double* b = (double*)malloc(sizeof(double) * vol);
  double* u = (double*)malloc(sizeof(double) * vol);
  if (!b || !u) return 1;
  double lam = 0.0;
  const int ks[3] = {k1, k2, k3};
  for (int a = 0; a < 3; ++a) {
    const double s = sin(kPi * ks[a] / (2.0 * (n + 1)));
    lam += 4.0 / (h * h) * s * s;
  }
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x)
        b[((size_t)z * n + y) * n + x] = sin(kPi * (double)((x + 1) * k1 % (2 * (n + 1))) / (n + 1)) *
                                         sin(kPi * (double)((y + 1) * k2 % (2 * (n + 1))) / (n + 1)) *
                                         sin(kPi * (double)((z + 1) * k3 % (2 * (n + 1))) / (n + 1));
  double *db = NULL, *du = NULL;
  HCHECK(hipMalloc((void**)&db, sizeof(double) * vol));
  HCHECK(hipMalloc((void**)&du, sizeof(double) * vol));
  HCHECK(hipMemcpy(db, b, sizeof(double) * vol, hipMemcpyHostToDevice));
  dpm_grid g = {n, h, sigma, x0};
  dpm_opts o = {DPM_FP64, 1, 1e-10, 0, 0, NULL, 0};
  size_t wsb = 0;
  CHECK(dpm_workspace_size(&g, 1, &o, &wsb));
  void* ws = NULL;
  HCHECK(hipMalloc(&ws, wsb > 0 ? wsb : 1));
  o.workspace = ws;
  o.workspace_bytes = wsb;
  CHECK(aux_solve(&g, db, du, &o, NULL, NULL));
  HCHECK(hipMemcpy(u, du, sizeof(double) * vol, hipMemcpyDeviceToHost));
  double err = 0.0, mx = 0.0;
  for (size_t i = 0; i < vol; ++i) {
    const double ref = b[i] / (sigma + lam);
    err = fmax(err, fabs(u[i] - ref));
    mx = fmax(mx, fabs(ref));
  }
  printf("sine mode n=%d rel err %.2e\n", n, err / mx);
  if (!(err <= 1e-12 * mx)) return 1;

  /* ---- 2. argument checks: nothing is launched, the error text names the problem */
  dpm_grid bad = {700, h, sigma, x0};  /* beyond every transform's sizes: rejected before launch */
  if (aux_solve(&bad, db, du, &o, NULL, NULL) != DPM_EINVAL) return 1;
  printf("n = 700 rejected: %s\n", dpm_last_error());
  dpm_grid negs = {n, h, -1.0, x0};
  if (aux_solve(&negs, db, du, &o, NULL, NULL) != DPM_EINVAL) return 1;

  /* ---- 3. DPM time loop on the unit sphere (l <= 2, beta = 1: 18 densities) */
  const double dt = 0.5 * h * h;
  dpm_grid gs = {n, h, 1.0 / dt, x0};
  dpm_geometry geo = {0, {0.0, 0.0, 0.0}, {1.0, 1.0, 1.0}};
  uint8_t* mp = NULL;
  HCHECK(hipMalloc((void**)&mp, vol));
  CHECK(dpm_classify(&gs, &geo, mp, NULL));
  int32_t ng = 0, ngi = 0;
  CHECK(dpm_gamma_points(&gs, mp, &ng, &ngi, NULL, NULL, NULL));
  int32_t* idx = NULL;
  uint8_t* is_in = NULL;
  HCHECK(hipMalloc((void**)&idx, sizeof(int32_t) * ng));
  HCHECK(hipMalloc((void**)&is_in, (size_t)ng));
  CHECK(dpm_gamma_points(&gs, mp, &ng, &ngi, idx, is_in, NULL));
  const int lmax = 2, nb = 2 * (lmax + 1) * (lmax + 1);
  double *basis = NULL, *dist = NULL;
  HCHECK(hipMalloc((void**)&basis, sizeof(double) * (size_t)nb * ng));
  HCHECK(hipMalloc((void**)&dist, sizeof(double) * ng));
  CHECK(dpm_basis(&gs, &geo, ng, idx, lmax, 1, basis, dist, NULL));
  dpm_bep* bep = NULL;
  CHECK(dpm_build_boundary_matrix(&gs, mp, nb, basis, &o, NULL, &bep, NULL));
  double *rho = NULL, *c = NULL;
  HCHECK(hipMalloc((void**)&rho, sizeof(double) * vol));
  HCHECK(hipMalloc((void**)&c, sizeof(double) * vol));
  const double c3[3] = {0.0, 0.0, 0.0};
  CHECK(dpm_gauss_state(bep, &geo, 10.0, 4.0, c3, rho, NULL));
  CHECK(dpm_gauss_state(bep, &geo, 5.0, 2.0, c3, c, NULL));
  dpm_opts so = {DPM_FP64, 1, 1e-10, 0, 0, NULL, 0};
  size_t swb = 0;
  CHECK(dpm_step_workspace_size(bep, &so, &swb));
  void* sws = NULL;
  HCHECK(hipMalloc(&sws, swb));
  so.workspace = sws;
  so.workspace_bytes = swb;
  dpm_stepper* st = NULL;
  CHECK(dpm_stepper_create(bep, dt, 1.0, rho, c, &so, NULL, &st));
  CHECK(dpm_stepper_run(st, 3, NULL));
  int32_t bad_step = -1;
  CHECK(dpm_stepper_first_nonfinite(st, NULL, &bad_step));
  HCHECK(hipMemcpy(u, rho, sizeof(double) * vol, hipMemcpyDeviceToHost));
  double mass = 0.0;
  for (size_t i = 0; i < vol; ++i) mass += u[i];
  printf("dpm: |gamma| = %d, |gamma_in| = %d, 3 captured steps, first non-finite step %d, "
         "sum rho %.6e\n", ng, ngi, bad_step, mass);
  if (bad_step != 0 || !(mass > 0.0) || !isfinite(mass)) return 1;
  dpm_stepper_destroy(st);

  /* ---- 4. adaptive loop (Steps 3-8) from Test A data: the CFL-type bound cuts dt below
   *         0.5 h^2 at the first step, which rebuilds the boundary matrix in place */
  size_t rwb = 0;
  CHECK(dpm_run_workspace_size(bep, &so, &rwb));
  void* rws = NULL;
  HCHECK(hipMalloc(&rws, rwb));
  dpm_opts ro = so;
  ro.workspace = rws;
  ro.workspace_bytes = rwb;
  CHECK(dpm_gauss_state(bep, &geo, 1000.0, 100.0, c3, rho, NULL));
  CHECK(dpm_gauss_state(bep, &geo, 500.0, 50.0, c3, c, NULL));
  const dpm_run_params rp = {1.0, 1.0, 1e30, 4};
  dpm_run_info ri;
  double dts[4];
  uint8_t rbs[4];
  CHECK(dpm_run(bep, &rp, rho, c, &ro, NULL, &ri, dts, rbs));
  printf("adaptive: %d steps, %d rebuilds, dt %.3e -> %.3e (0.5 h^2 = %.3e), stop %d, max rho %.3e\n",
         ri.steps, ri.rebuilds, dts[0], ri.dt, dt, ri.stop, ri.rho_max);
  if (ri.steps != 4 || ri.rebuilds < 1 || !rbs[0] || !(dts[0] < dt) || ri.stop != DPM_RUN_MAXSTEPS ||
      !isfinite(ri.rho_max))
    return 1;
  dpm_bep_destroy(bep);

  /* ---- 5. domain decomposition, Case 2: the cap |x - (0,0,1)| < 0.5 on its own 15^3 mesh of
   *         [-0.75, 0.75]^2 x [0, 1.5], the rest of the ball on the 31^3 mesh; Test B data;
   *         three adaptive steps of the coupled problem */
  const int n1 = 15;
  const double h1 = 1.5 / (n1 + 1);
  dpm_dd2_params dp = {{n1, h1, 1.0 / dt, -0.75 + h1}, {n, h, 1.0 / dt, x0}, {0.0, 0.0, 0.75},
                       {0.0, 0.0, 0.0}, 1.0, 1.0, 0.5, 2.0, 4, 0, 2};
  dpm_dd* dd = NULL;
  CHECK(dpm_dd2_build(&dp, &o, NULL, &dd, NULL));
  int32_t dg[2], dgi[2], drows[2], dcols = 0;
  CHECK(dpm_dd_info(dd, dg, dgi, drows, &dcols, NULL, NULL));
  const size_t vol1 = (size_t)n1 * n1 * n1;
  double* st4[4] = {NULL, NULL, NULL, NULL};
  HCHECK(hipMalloc((void**)&st4[0], sizeof(double) * vol1));
  HCHECK(hipMalloc((void**)&st4[1], sizeof(double) * vol1));
  HCHECK(hipMalloc((void**)&st4[2], sizeof(double) * vol));
  HCHECK(hipMalloc((void**)&st4[3], sizeof(double) * vol));
  const double cb[3] = {0.0, 0.0, 0.25};
  for (int l = 0; l < 2; ++l) {
    CHECK(dpm_dd_gauss_state(dd, l, 2000.0, 100.0, cb, st4[2 * l], NULL));
    CHECK(dpm_dd_gauss_state(dd, l, 0.0, 1.0, cb, st4[2 * l + 1], NULL));
  }
  size_t dwb = 0;
  CHECK(dpm_dd_run_workspace_size(dd, &so, &dwb));
  void* dws = NULL;
  HCHECK(hipMalloc(&dws, dwb));
  dpm_opts dop = so;
  dop.workspace = dws;
  dop.workspace_bytes = dwb;
  const dpm_run_params dr = {1.0, 1.0, 1e30, 3};
  dpm_run_info di;
  CHECK(dpm_dd_run(dd, &dr, st4, &dop, NULL, &di, NULL, NULL));
  double* h1v = (double*)malloc(sizeof(double) * vol1);
  if (!h1v) return 1;
  HCHECK(hipMemcpy(h1v, st4[0], sizeof(double) * vol1, hipMemcpyDeviceToHost));
  double m1 = 0.0;
  for (size_t i = 0; i < vol1; ++i) m1 += h1v[i];
  printf("dd case 2: rows %d + %d, %d columns, %d steps, %d rebuilds, max rho %.3e, sum rho_1 %.6e\n",
         drows[0], drows[1], dcols, di.steps, di.rebuilds, di.rho_max, m1);
  if (di.steps != 3 || !(m1 > 0.0) || !isfinite(m1) || !isfinite(di.rho_max) || drows[0] <= dgi[0])
    return 1;
  dpm_dd_destroy(dd);
  free(h1v);
  (void)hipFree(dws);
  for (int i = 0; i < 4; ++i) (void)hipFree(st4[i]);
  (void)hipFree(rws);
  (void)hipFree(sws); (void)hipFree(rho); (void)hipFree(c); (void)hipFree(basis);
  (void)hipFree(dist); (void)hipFree(idx); (void)hipFree(is_in); (void)hipFree(mp);
  (void)hipFree(ws); (void)hipFree(db); (void)hipFree(du);
  free(b);
  free(u);
  printf("ok\n");
  return 0;
}
