// Covariance models in FP64 (device side). GSLIB convention: total sill,
// practical range a; Cov(0) = sill, Cov(h > 0) = (sill - nugget) rho(h) with
//   spherical   rho = 1 - 1.5 h/a + 0.5 (h/a)^3 for h < a, else 0
//   exponential rho = exp(-3 h / a)
//   Gaussian    rho = exp(-3 h^2 / a^2)
// and the derivatives of Cov with respect to (nugget, sill, range).
#pragma once

#include "okrig_internal.h"

namespace okr {

__device__ inline double rho_d(int model, double h, double a) {
  if (model == 0) {
    double q = h / a;
    return q < 1.0 ? 1.0 - 1.5 * q + 0.5 * q * q * q : 0.0;
  }
  if (model == 1) return exp(-3.0 * h / a);
  double q = h / a;
  return exp(-3.0 * q * q);
}

__device__ inline double drho_da_d(int model, double h, double a) {
  if (model == 0) {
    double q = h / a;
    return q < 1.0 ? 1.5 * h / (a * a) - 1.5 * h * h * h / (a * a * a * a) : 0.0;
  }
  if (model == 1) return exp(-3.0 * h / a) * 3.0 * h / (a * a);
  double q = h / a;
  return exp(-3.0 * q * q) * 6.0 * h * h / (a * a * a);
}

__device__ inline double cov_d(const Vario& v, double h) {
  return h == 0.0 ? v.sill : (v.sill - v.nugget) * rho_d(v.model, h, v.range);
}

__device__ inline void cov_and_grad(const Vario v, double h, double* c, double* dn, double* ds,
                                    double* da) {
  if (h == 0.0) {
    *c = v.sill; *dn = 0.0; *ds = 1.0; *da = 0.0;
    return;
  }
  double rho = rho_d(v.model, h, v.range);
  *c = (v.sill - v.nugget) * rho;
  *dn = -rho;
  *ds = rho;
  *da = (v.sill - v.nugget) * drho_da_d(v.model, h, v.range);
}

}  // namespace okr
