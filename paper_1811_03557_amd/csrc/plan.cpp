// Per-(device, n) tables of the sine transforms: the packed sine/twiddle table of the real-FFT
// DST-I, the 1D Dirichlet eigenvalues and the split-bf16 dense sine matrix.  Computed on the host in FP64 from their definitions
// (std::sin / std::cos), uploaded once and kept until the process ends.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>

#include "common.h"

namespace dpm {

namespace {
thread_local std::string g_err;
std::mutex g_plan_mu;
std::map<std::pair<int, int>, Plan*> g_plans;

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
}  // namespace

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error_text() { return g_err.c_str(); }

bool fft_size_supported(int n) {
  if (n < 7 || n > 1023) return false;
  int m = n + 1;
  return (m & (m - 1)) == 0;
}

bool dense_size_supported(int n) { return n >= 7 && n <= kDenseMaxN; }

// Bluestein tables of the DST-I of length n (M = n + 1): the chirp w_j = e^{i pi j^2/(2M)} with
// the phase reduced exactly (j^2 mod 4M), the filter c_d = conj(w_|d|) at d mod L for
// 1 - n <= d <= 2M - 2, its DFT divided by L (direct sum in long double), and the FFT twiddles.
static dpm_status build_blue(int n, Plan* p) {
  const int lg = blue_logl(n);
  const int L = 1 << lg, M = n + 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  auto chirp = [&](long long d) {  // e^{i pi d^2 / (2M)}
    const long long r = (d * d) % (4LL * M);
    const long double a = pi * (long double)r / (2.0L * (long double)M);
    return std::make_pair(std::cos(a), std::sin(a));
  };
  std::vector<double> tw(2 * (size_t)L), w(2 * (size_t)(M + 1)), ch(2 * (size_t)L);
  std::vector<long double> cr(L, 0.0L), ci(L, 0.0L), tr(L), ti(L);
  for (int e = 0; e < L; ++e) {
    const long double a = -2.0L * pi * (long double)e / (long double)L;
    tr[e] = std::cos(a);
    ti[e] = std::sin(a);
    tw[2 * e] = (double)tr[e];
    tw[2 * e + 1] = (double)ti[e];
  }
  for (int j = 0; j <= M; ++j) {
    const auto c = chirp(j);
    w[2 * j] = (double)c.first;
    w[2 * j + 1] = (double)c.second;
  }
  for (long long d = 1 - n; d <= 2LL * M - 2; ++d) {
    const auto c = chirp(d < 0 ? -d : d);
    const int pos = (int)(((d % L) + L) % L);
    cr[pos] = c.first;
    ci[pos] = -c.second;  // conj
  }
  for (int k = 0; k < L; ++k) {
    long double sr = 0.0L, si = 0.0L;
    for (int q = 0; q < L; ++q) {
      const int e = (int)(((long long)q * k) % L);
      sr += cr[q] * tr[e] - ci[q] * ti[e];
      si += cr[q] * ti[e] + ci[q] * tr[e];
    }
    ch[2 * k] = (double)(sr / (long double)L);
    ch[2 * k + 1] = (double)(si / (long double)L);
  }
  p->blue_logl = lg;
  DPM_TRY_HIP(hipMalloc(&p->blue_tw, sizeof(double) * tw.size()));
  DPM_TRY_HIP(hipMalloc(&p->blue_w, sizeof(double) * w.size()));
  DPM_TRY_HIP(hipMalloc(&p->blue_ch, sizeof(double) * ch.size()));
  DPM_TRY_HIP(hipMemcpy(p->blue_tw, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->blue_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->blue_ch, ch.data(), sizeof(double) * ch.size(), hipMemcpyHostToDevice));
  return DPM_OK;
}

static dpm_status build_plan(int n, Plan* p) {
  p->n = n;
  const int M = n + 1;
  const int L = 2 * M;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  p->log2L = lg;
  const double pi = std::acos(-1.0);
  // packed transform table: [ sin(pi j/M), j < M | e^{-2 pi i e/H}, e < H | e^{-2 pi i k/M}, k < H ]
  const int H = M / 2;
  std::vector<double> tabd(3 * (size_t)M);
  for (int j = 0; j < M; ++j) tabd[j] = std::sin(pi * (double)j / (double)M);
  for (int e = 0; e < H; ++e) {
    const double a = -2.0 * pi * (double)e / (double)H;
    tabd[M + 2 * e] = std::cos(a);
    tabd[M + 2 * e + 1] = std::sin(a);
  }
  for (int k = 0; k < H; ++k) {
    const double a = -2.0 * pi * (double)k / (double)M;
    tabd[2 * M + 2 * k] = std::cos(a);
    tabd[2 * M + 2 * k + 1] = std::sin(a);
  }
  std::vector<float> tabf(tabd.size());
  for (size_t i = 0; i < tabd.size(); ++i) tabf[i] = (float)tabd[i];
  std::vector<double> lam(n);
  for (int k = 1; k <= n; ++k) {
    double s = std::sin(pi * k / (2.0 * M));
    lam[k - 1] = 4.0 * s * s;
  }
  // dense orthonormal DST-I matrix padded to a multiple of 32, split into bf16 hi + lo
  int mpad = (n + 31) / 32 * 32;
  std::vector<uint16_t> hi((size_t)mpad * mpad, 0), lo((size_t)mpad * mpad, 0);
  const bool dense64 = dense_size_supported(n);
  std::vector<double> sd(dense64 ? (size_t)mpad * mpad : 0, 0.0);
  const double nrm = std::sqrt(2.0 / M);
  for (int j = 1; j <= n; ++j)
    for (int k = 1; k <= n; ++k) {
      double v = nrm * std::sin(pi * (double)j * (double)k / (double)M);
      float vf = (float)v;
      uint16_t h = bf16_rne(vf);
      float r = (float)(v - (double)bf16_to_f(h));
      hi[(size_t)(j - 1) * mpad + (k - 1)] = h;
      lo[(size_t)(j - 1) * mpad + (k - 1)] = bf16_rne(r);
      if (dense64) sd[(size_t)(j - 1) * mpad + (k - 1)] = v;
    }
  p->mpad = mpad;
  DPM_TRY_HIP(hipMalloc(&p->tw_f, sizeof(float) * tabf.size()));
  DPM_TRY_HIP(hipMalloc(&p->tw_d, sizeof(double) * tabd.size()));
  DPM_TRY_HIP(hipMalloc(&p->lam, sizeof(double) * n));
  DPM_TRY_HIP(hipMalloc(&p->s_hi, sizeof(uint16_t) * hi.size()));
  DPM_TRY_HIP(hipMalloc(&p->s_lo, sizeof(uint16_t) * lo.size()));
  DPM_TRY_HIP(hipMemcpy(p->tw_f, tabf.data(), sizeof(float) * tabf.size(), hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->tw_d, tabd.data(), sizeof(double) * tabd.size(), hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->lam, lam.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->s_hi, hi.data(), sizeof(uint16_t) * hi.size(), hipMemcpyHostToDevice));
  DPM_TRY_HIP(hipMemcpy(p->s_lo, lo.data(), sizeof(uint16_t) * lo.size(), hipMemcpyHostToDevice));
  if (dense64) {
    DPM_TRY_HIP(hipMalloc(&p->s_d, sizeof(double) * sd.size()));
    DPM_TRY_HIP(hipMemcpy(p->s_d, sd.data(), sizeof(double) * sd.size(), hipMemcpyHostToDevice));
  }
  if (blue_size_supported(n)) DPM_TRY(build_blue(n, p));
  return DPM_OK;
}

dpm_status get_plan(int n, const Plan** out) {
  int dev = 0;
  DPM_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto key = std::make_pair(dev, n);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
    return DPM_OK;
  }
  Plan* p = new Plan();
  dpm_status st = build_plan(n, p);
  if (st != DPM_OK) {
    (void)hipFree(p->tw_f);
    (void)hipFree(p->tw_d);
    (void)hipFree(p->lam);
    (void)hipFree(p->s_hi);
    (void)hipFree(p->s_lo);
    (void)hipFree(p->s_d);
    (void)hipFree(p->blue_tw);
    (void)hipFree(p->blue_w);
    (void)hipFree(p->blue_ch);
    delete p;
    return st;
  }
  g_plans[key] = p;
  *out = p;
  return DPM_OK;
}

dpm_status find_plan(int n, const Plan** out) {
  int dev = 0;
  DPM_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(std::make_pair(dev, n));
  if (it == g_plans.end()) {
    set_error("the tables of n = %d are not built on device %d: call dpm_prepare(%d) first", n,
              dev, n);
    return DPM_EINVAL;
  }
  *out = it->second;
  return DPM_OK;
}

}  // namespace dpm
