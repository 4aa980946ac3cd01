// Bessel functions of the first kind J_m(tau), 0 <= m < Np, for the
// Chebyshev-Bessel expansion of the evolution operator (Section 3.2).
//
// Method: Miller's backward recurrence (J. C. P. Miller, British Association
// Mathematical Tables, 1952; see Abramowitz & Stegun 9.12): start far above
// both Np and tau with an arbitrary tiny seed, run
//     j_{k-1} = (2k / tau) j_k - j_{k+1}
// downwards (stable in that direction for every k), and normalise with the
// sum rule J_0 + 2 (J_2 + J_4 + ...) = 1.  Values are rescaled whenever they
// grow past 1e250, so nothing overflows for large orders.
//
// Compiled for both host (coefficient counts, host helper) and device (the
// per-segment coefficient table kernel).
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define GPUQT_HD __host__ __device__
#else
#define GPUQT_HD
#endif

// Starting order: far enough above max(Np, tau) that the seed error has
// decayed below double precision by the time the recurrence reaches Np.
GPUQT_HD inline int bessel_start_order(double tau, int Np) {
  double top = tau > (double)Np ? tau : (double)Np;
  int m = (int)(top + 30.0 + 12.0 * cbrt(top + 1.0) + sqrt(40.0 * (top + 1.0)));
  return m + (m & 1);  // even
}

// J[m] = J_m(tau) for m < Np.  tau >= 0.
GPUQT_HD inline void bessel_miller(double tau, int Np, double* J) {
  if (Np <= 0) return;
  if (tau == 0.0) {
    J[0] = 1.0;
    for (int m = 1; m < Np; ++m) J[m] = 0.0;
    return;
  }
  const int top = bessel_start_order(tau, Np);
  double jp1 = 0.0;     // j_{k+1}
  double jk = 1e-280;   // j_k, arbitrary seed at k = top
  double sum = 0.0;     // J_0 + 2 * sum of even orders, unnormalised
  for (int m = 0; m < Np; ++m) J[m] = 0.0;
  for (int k = top; k >= 1; --k) {
    if (k < Np) J[k] = jk;
    if ((k & 1) == 0) sum += 2.0 * jk;
    const double jm1 = (2.0 * k / tau) * jk - jp1;
    jp1 = jk;
    jk = jm1;
    if (fabs(jk) > 1e250) {
      const double s = 1e-250;
      jk *= s;
      jp1 *= s;
      sum *= s;
      const int lo = k;  // stored orders >= k
      for (int m = lo; m < Np; ++m) J[m] *= s;
    }
  }
  // jk now holds j_0
  sum += jk;
  J[0] = jk;
  const double inv = 1.0 / sum;
  for (int m = 0; m < Np; ++m) J[m] *= inv;
}
