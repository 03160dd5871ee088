// Per-particle material update (the operator M^-1 of Sec. 3.2), shared by
// the single-problem and batched Newton steps.
//
// Solves u(e) = rho/dt (e - e^{n-1}) + c sigma_a a (e/c_v)^4 - P = 0 with
// P = Q_e + c sigma_a E^{l+1}, by Newton with J = rho/dt + 4 c sigma_a a T^3/c_v,
// T = e/c_v.  u is increasing and convex on e >= 0 with u(0) <= 0 <=
// u(e^{n-1} + dt P/rho), so a Newton step leaving the current bracket is
// replaced by bisection; a negative upper end means the root is negative
// (reported as non-physical, e clamped to 0).
#pragma once

#include <cmath>

namespace rt {

struct MaterialResult {
  double e;
  int iterations;
  bool converged;
  bool nonphysical;
};

__device__ __forceinline__ MaterialResult material_solve(double rho, double cv, double sa,
                                                         double ep, double Qe, double Enew,
                                                         double e_start, double dt, double c,
                                                         double a, double tol, int max_iter) {
  const double ca = c * sa;
  const double P = Qe + ca * Enew;
  const double rdt = rho / dt;
  double lo = 0.0, hi = ep + dt * P / rho;
  MaterialResult res{0.0, 0, true, false};
  if (hi < 0.0) {
    res.nonphysical = true;
    return res;
  }
  double e = fmin(fmax(e_start, lo), hi);
  res.converged = false;
  int it = 0;
  while (it < max_iter) {
    const double T = e / cv;
    const double T2 = T * T;
    const double u = rdt * (e - ep) + ca * a * (T2 * T2) - P;
    const double J = rdt + 4.0 * ca * a * (T2 * T) / cv;
    ++it;
    if (u == 0.0) {
      res.converged = true;
      break;
    }
    if (u > 0.0) hi = e;
    else lo = e;
    const double en = e - u / J;
    const bool small = fabs(en - e) <= tol * fabs(en);
    const bool inside = en > lo && en < hi;
    e = (small || inside) ? en : 0.5 * (lo + hi);
    if (small) {
      res.converged = true;
      break;
    }
  }
  res.e = e;
  res.iterations = it;
  return res;
}

}  // namespace rt
