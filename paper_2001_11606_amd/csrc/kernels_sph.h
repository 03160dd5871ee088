// Device-side SPH kernel derivatives (Sec. 2.3) for dim in {2, 3}.
//   cubic B-spline (support 2h):  W = s_d h^-d w(q), w' = -3q + 9/4 q^2 (q < 1),
//                                 -3/4 (2 - q)^2 (1 <= q < 2); s_2 = 10/(7 pi), s_3 = 1/pi
//   Wendland C4 (support h):      W = k_d h^-d (1-q)^5 (8q^2 + 5q + 1),
//                                 dpsi/dq = -14 q (4q + 1)(1 - q)^4;
//                                 k_2 = 36/(5 pi), k_3 = 45/(4 pi) from the
//                                 normalisation condition of Sec. 2.3.
#pragma once

#include <hip/hip_runtime.h>

namespace rt {

constexpr double kPi = 3.14159265358979323846;

template <int DIM>
__device__ __forceinline__ double sph_dwdr(double r, double h, int kernel) {
  const double hinv = 1.0 / h;
  const double q = r * hinv;
  double hpow = hinv * hinv * hinv;          // h^-(dim+1)
  if (DIM == 3) hpow *= hinv;
  if (kernel == RT_KERNEL_CUBIC_SPLINE) {
    const double sig = DIM == 2 ? 10.0 / (7.0 * kPi) : 1.0 / kPi;
    double dw = 0.0;
    if (q < 1.0) dw = -3.0 * q + 2.25 * q * q;
    else if (q < 2.0) dw = -0.75 * (2.0 - q) * (2.0 - q);
    return sig * dw * hpow;
  }
  const double k = DIM == 2 ? 36.0 / (5.0 * kPi) : 45.0 / (4.0 * kPi);
  double dw = 0.0;
  if (q < 1.0) {
    const double om = 1.0 - q;
    const double om2 = om * om;
    dw = -14.0 * q * (4.0 * q + 1.0) * (om2 * om2);
  }
  return k * dw * hpow;
}

}  // namespace rt
