// Device-side geometry shared by the geometry and DPM kernels: the domain descriptor, the
// inside predicate of M+ and the projection of a node onto Gamma.
#pragma once

#include "common.h"

namespace dpm {

struct GeoDev {
  int kind;
  double cx, cy, cz;
  double a, b, c;
};

inline GeoDev to_dev(const dpm_geometry& g) {
  GeoDev d;
  d.kind = g.kind;
  d.cx = g.center[0];
  d.cy = g.center[1];
  d.cz = g.center[2];
  d.a = g.axes[0];
  d.b = g.kind == 0 ? g.axes[0] : g.axes[1];
  d.c = g.kind == 0 ? g.axes[0] : g.axes[2];
  return d;
}

__device__ __forceinline__ bool inside(const GeoDev& g, double x, double y, double z) {
  const double px = x - g.cx, py = y - g.cy, pz = z - g.cz;
  if (g.kind == 0) return px * px + py * py + pz * pz < g.a * g.a;
  const double u = px / g.a, v = py / g.b, w = pz / g.c;
  return u * u + v * v + w * w < 1.0;
}

// ------------------------------------------------------------------ projection onto Gamma
// Closest point q of Gamma to p (relative to the centre); returns d (+ outside) and the
// polar/azimuthal angles of q (parametric angles for the ellipsoid).
// q3 (nullable) receives the foot point relative to the centre.
__device__ inline void project(const GeoDev& g, double px, double py, double pz, double* d,
                               double* th, double* ph, double* q3 = nullptr) {
  if (g.kind == 0) {
    const double r = sqrt(px * px + py * py + pz * pz);
    *d = r - g.a;
    *th = atan2(sqrt(px * px + py * py), pz);  // well conditioned at the poles
    *ph = atan2(py, px);
    if (q3) {
      const double f = r > 0.0 ? g.a / r : 0.0;
      q3[0] = f * px;
      q3[1] = f * py;
      q3[2] = r > 0.0 ? f * pz : g.a;
    }
    return;
  }
  // ellipsoid: q_i = a_i^2 p_i / (a_i^2 + t), t the root of
  // F(t) = sum a_i^2 p_i^2 / (a_i^2 + t)^2 - 1 on (-min a_i^2, inf), by safeguarded Newton
  const double a2 = g.a * g.a, b2 = g.b * g.b, c2 = g.c * g.c;
  const double m2 = fmin(a2, fmin(b2, c2));
  const double lev = px * px / a2 + py * py / b2 + pz * pz / c2;
  double lo, hi;
  if (lev > 1.0) {
    lo = 0.0;
    hi = 1.0;
    for (int it = 0; it < 200; ++it) {
      const double fa = a2 * px / (a2 + hi), fb = b2 * py / (b2 + hi), fc = c2 * pz / (c2 + hi);
      if ((fa * fa) / a2 + (fb * fb) / b2 + (fc * fc) / c2 < 1.0) break;
      hi *= 2.0;
    }
  } else {
    lo = -m2 * (1.0 - 1e-15);
    hi = 0.0;
  }
  double t = lev > 1.0 ? 0.0 : 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double da = a2 + t, db = b2 + t, dc = c2 + t;
    const double qa = a2 * px * px / (da * da), qb = b2 * py * py / (db * db), qc = c2 * pz * pz / (dc * dc);
    const double F = qa + qb + qc - 1.0;
    const double dF = -2.0 * (qa / da + qb / db + qc / dc);
    if (F > 0.0) lo = t; else hi = t;
    double tn = (dF != 0.0) ? t - F / dF : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (fabs(tn - t) <= 1e-16 * fmax(1.0, fabs(t)) || hi - lo <= 1e-16 * fmax(1.0, fabs(t))) {
      t = tn;
      break;
    }
    t = tn;
  }
  const double qx = a2 * px / (a2 + t), qy = b2 * py / (b2 + t), qz = c2 * pz / (c2 + t);
  if (q3) {
    q3[0] = qx;
    q3[1] = qy;
    q3[2] = qz;
  }
  const double dist = sqrt((px - qx) * (px - qx) + (py - qy) * (py - qy) + (pz - qz) * (pz - qz));
  *d = lev > 1.0 ? dist : -dist;
  const double u = qx / g.a, v = qy / g.b, w = qz / g.c;
  *th = atan2(sqrt(u * u + v * v), w);  // parametric polar angle, well conditioned at the poles
  *ph = atan2(v, u);
}


}  // namespace dpm
