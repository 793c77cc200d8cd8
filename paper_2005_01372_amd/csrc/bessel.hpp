// FP64 Bessel functions for the cell-integrated Green's function table.
//
// The table needs H0^(1)(x) = J0(x) + i Y0(x) for x in [k0 h, k0 h sqrt(nx^2+nz^2)]
// and, for the self cell, J1 and H1^(1) at the small argument k0 a.
//
//  * 0 < x < 20: J_n by Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1},
//    normalised with J0 + 2 sum_k J_{2k} = 1, and Y0 from the Neumann series
//    (pi/2) Y0 = (ln(x/2) + gamma) J0 - 2 sum_{k>=1} (-1)^k J_{2k} / k
//    (Abramowitz & Stegun 9.1.46 and 9.1.88).
//  * x >= 20: Hankel's asymptotic expansion
//    H0^(1)(x) = sqrt(2/(pi x)) e^{i(x - pi/4)} sum_k i^k a_k / x^k,
//    a_k = a_{k-1} (-(2k-1)^2) / (8k) (A&S 9.2.5-9.2.10); the smallest term is
//    about e^{-2x}, below double rounding for x >= 20.
//  * J1, Y1 at small x (x <= 2): ascending series (A&S 9.1.10, 9.1.11).
#pragma once
#include <math.h>
#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#else
#define __host__
#define __device__
#endif

namespace lsop_bessel {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.577215664901532860606512090082402431;

// H0^(1)(x) for x > 0; returns (J0, Y0).
__host__ __device__ inline void hankel0(double x, double* j0, double* y0) {
  if (x < 20.0) {
    // backward recurrence from an even start order well above x
    int m = 2 * (int)((x + 30.0 + 4.0 * sqrt(x)) * 0.5);
    double jp1 = 0.0, jn = 1e-30;  // J_{m+1}, J_m (unnormalised)
    double sum_even = 0.0;          // J0 + 2 sum J_{2k}, accumulated below
    double neu = 0.0;               // sum_{k>=1} (-1)^k J_{2k} / k
    double j_0 = 0.0;
    for (int n = m; n >= 1; --n) {
      if ((n & 1) == 0) {
        sum_even += 2.0 * jn;
        const int k = n / 2;
        neu += ((k & 1) ? -jn : jn) / (double)k;
      }
      const double jm1 = (2.0 * n / x) * jn - jp1;
      jp1 = jn;
      jn = jm1;
      if (fabs(jn) > 1e250) {  // rescale to stay in range
        jn *= 1e-250;
        jp1 *= 1e-250;
        sum_even *= 1e-250;
        neu *= 1e-250;
      }
    }
    j_0 = jn;
    sum_even += j_0;
    const double s = 1.0 / sum_even;
    *j0 = j_0 * s;
    *y0 = (2.0 / kPi) * ((log(0.5 * x) + kEulerGamma) * (*j0) - 2.0 * neu * s);
    return;
  }
  // asymptotic expansion: sum_k i^k a_k x^-k = P + i Q
  double P = 1.0, Q = 0.0, a = 1.0, xk = 1.0;
  const double inv = 1.0 / x;
  for (int k = 1; k < 60; ++k) {
    a *= -(double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k);
    xk *= inv;
    const double t = a * xk;
    switch (k & 3) {  // i^k
      case 0: P += t; break;
      case 1: Q += t; break;
      case 2: P -= t; break;
      default: Q -= t; break;
    }
    if (fabs(t) < 1e-17) break;
  }
  double sx, cx;
  sincos(x, &sx, &cx);
  // e^{i(x - pi/4)} = (cos x + i sin x)(1 - i)/sqrt2
  const double r2 = 0.707106781186547524400844362104849039;
  const double er = r2 * (cx + sx), ei = r2 * (sx - cx);
  const double amp = sqrt(2.0 / (kPi * x));
  *j0 = amp * (er * P - ei * Q);
  *y0 = amp * (er * Q + ei * P);
}

// J1 and Y1 for 0 < x <= 2 by their ascending series.
__host__ __device__ inline void bessel1_small(double x, double* j1, double* y1) {
  const double hx = 0.5 * x, q = -hx * hx;
  double term = hx;  // (x/2)^{2k+1} (-1)^k / (k! (k+1)!) at k = 0
  double sj = 0.0, sy = 0.0;
  double psi_k1 = -kEulerGamma;            // psi(k+1)
  double psi_k2 = -kEulerGamma + 1.0;      // psi(k+2)
  for (int k = 0; k < 40; ++k) {
    sj += term;
    sy += (psi_k1 + psi_k2) * term;
    term *= q / ((double)(k + 1) * (double)(k + 2));
    psi_k1 += 1.0 / (k + 1);
    psi_k2 += 1.0 / (k + 2);
    if (fabs(term) < 1e-18 * fabs(sj)) break;
  }
  *j1 = sj;
  *y1 = -2.0 / (kPi * x) + (2.0 / kPi) * log(hx) * sj - sy / kPi;
}

}  // namespace lsop_bessel
