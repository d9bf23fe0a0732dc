// The error bounds of section "Error estimates and conditioning", assembled
// on the host from the three sums the residual kernel returns.
#pragma once

#include <cmath>

#include "condest.h"

namespace condest {

// sums = (||A x_hat - b||^2, ||x_hat||^2, ||b||^2). Returns COND_ENUMERIC when
// b or x_hat is zero or a sum is not finite.
inline int fill_bounds(const double* sums, double kappa, double norm_a, cond_bounds_t* out) {
  constexpr double kEpsMach = 2.220446049250313e-16;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(sums[k])) return COND_ENUMERIC;
  if (!(sums[1] > 0.0) || !(sums[2] > 0.0)) return COND_ENUMERIC;
  const double inf = HUGE_VAL;
  cond_bounds_t r{};
  r.res_norm = std::sqrt(sums[0]);
  r.x_norm = std::sqrt(sums[1]);
  r.b_norm = std::sqrt(sums[2]);
  r.rel_residual = r.res_norm / r.b_norm;
  // Theorem "Bounds on the relative error ||x_hat - x|| / ||x||"
  r.err_x_lower = r.rel_residual / kappa;
  r.err_x_upper = kappa * r.rel_residual;
  // Theorem "Bounds on the relative error ||x_hat - x|| / ||x_hat||"; the
  // upper bound is the epsilon of the next theorem
  r.err_xhat_lower = r.res_norm / (norm_a * r.x_norm);
  const double eps = kappa * r.res_norm / (norm_a * r.x_norm);
  r.err_xhat_upper = eps;
  // Theorem "Tight upper bound of the error ||x_hat - x|| / ||x||"
  r.err_x_tight = eps < 1.0 ? eps / (1.0 - eps) : inf;
  // Theorem "Numerical singularity of a matrix"
  r.roundoff_floor = kappa * kEpsMach < 1.0 ? 2.0 * kEpsMach * kappa / (1.0 - kappa * kEpsMach) : inf;
  *out = r;
  return COND_OK;
}

}  // namespace condest
