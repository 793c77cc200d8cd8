// FP64 Bessel functions of complex argument for the kernel table of a dissipative background (complex
// wavenumber k with Re k > 0, Im k >= 0).  The same methods as the real routines of bessel.hpp, in complex
// arithmetic:
//  * |z| + Im z < 20: J_n by Miller's backward recurrence, normalised with J0 + 2 sum_k J_{2k} = 1 (an identity of the
//    generating function, valid for complex z), and Y0 from the Neumann series
//    (pi/2) Y0 = (log(z/2) + gamma) J0 - 2 sum_{k>=1} (-1)^k J_{2k} / k with the principal logarithm
//    (Abramowitz & Stegun 9.1.46, 9.1.88);
//  * |z| + Im z >= 20: Hankel's expansion H0^(1)(z) = sqrt(2/(pi z)) e^{i(z - pi/4)} sum_k i^k a_k z^{-k},
//    a_k = a_{k-1} (-(2k-1)^2) / (8k), valid for |arg z| < pi (A&S 9.2.5-9.2.10).  The switch weighs the two
//    errors: the series forms H0 ~ e^{-Im z} as J0 + i Y0 with J0, Y0 ~ e^{Im z}, an absolute error near
//    1e-16 e^{Im z}; the expansion, summed up to its smallest term, has a relative error of about e^{-2|z|},
//    an absolute e^{-2|z| - Im z}; they cross at |z| + Im z ~ 18.4;
//  * J1, Y1 for |z| <= 2 by their ascending series (A&S 9.1.10, 9.1.11).
#pragma once
#include "bessel.hpp"
#include "cx.hpp"

namespace lsop_bessel {

using C = Cx<double>;

__host__ __device__ inline C c_div(C a, C b) {
  const double d = b.re * b.re + b.im * b.im;
  return C{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__host__ __device__ inline C c_log(C z) { return C{log(sqrt(z.re * z.re + z.im * z.im)), atan2(z.im, z.re)}; }
__host__ __device__ inline C c_sqrt(C z) {
  const double r = sqrt(z.re * z.re + z.im * z.im);
  const double s = sqrt(0.5 * (r + z.re)), t = sqrt(0.5 * fmax(r - z.re, 0.0));
  return C{s, z.im < 0 ? -t : t};
}
// e^{i z}
__host__ __device__ inline C c_expi(C z) {
  const double m = exp(-z.im);
  double sn, cs;
  sincos(z.re, &sn, &cs);
  return C{m * cs, m * sn};
}
__host__ __device__ inline double c_abs(C z) { return sqrt(z.re * z.re + z.im * z.im); }

// H0^(1)(z) = J0(z) + i Y0(z), Re z > 0.
__host__ __device__ inline C hankel0_c(C z) {
  const double az = c_abs(z);
  if (az + z.im < 20.0) {
    const int m = 2 * (int)((az + 30.0 + 4.0 * sqrt(az)) * 0.5);
    const C two_over_z = c_div(C{2.0, 0.0}, z);
    C jp1{0.0, 0.0}, jn{1e-30, 0.0};
    C sum_even{0.0, 0.0}, neu{0.0, 0.0};
    for (int n = m; n >= 1; --n) {
      if ((n & 1) == 0) {
        sum_even = sum_even + 2.0 * jn;
        const int k = n / 2;
        const double sg = (k & 1) ? -1.0 / k : 1.0 / k;
        neu = neu + sg * jn;
      }
      const C jm1 = (double)n * (two_over_z * jn) - jp1;
      jp1 = jn;
      jn = jm1;
      if (c_abs(jn) > 1e250) {
        jn = 1e-250 * jn;
        jp1 = 1e-250 * jp1;
        sum_even = 1e-250 * sum_even;
        neu = 1e-250 * neu;
      }
    }
    sum_even = sum_even + jn;
    const C j0 = c_div(jn, sum_even);
    const C nn = c_div(neu, sum_even);
    const C lg = c_log(0.5 * z) + C{kEulerGamma, 0.0};
    const C y0 = (2.0 / kPi) * (lg * j0 - 2.0 * nn);
    return C{j0.re - y0.im, j0.im + y0.re};
  }
  const C inv = c_div(C{1.0, 0.0}, z);
  C S{1.0, 0.0}, zk{1.0, 0.0};
  double a = 1.0, prev = 1.0;
  for (int k = 1; k < 60; ++k) {
    a *= -(double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k);
    zk = zk * inv;
    C t = a * zk;
    const double at = c_abs(t);
    if (at > prev) break;  // the expansion diverges past its smallest term (near k = 2|z|)
    prev = at;
    switch (k & 3) {  // times i^k
      case 1: t = C{-t.im, t.re}; break;
      case 2: t = C{-t.re, -t.im}; break;
      case 3: t = C{t.im, -t.re}; break;
      default: break;
    }
    S = S + t;
    if (c_abs(t) < 1e-17 * c_abs(S)) break;
  }
  const C amp = c_sqrt(c_div(C{2.0 / kPi, 0.0}, z));
  const C ph = c_expi(z - C{0.25 * kPi, 0.0});
  return amp * ph * S;
}

// J1(z) and Y1(z) for |z| <= 2.
__host__ __device__ inline void bessel1_small_c(C z, C* j1, C* y1) {
  const C hx = 0.5 * z;
  const C q = -1.0 * (hx * hx);
  C term = hx;
  C sj{0.0, 0.0}, sy{0.0, 0.0};
  double psi_k1 = -kEulerGamma, psi_k2 = -kEulerGamma + 1.0;
  for (int k = 0; k < 40; ++k) {
    sj = sj + term;
    sy = sy + (psi_k1 + psi_k2) * term;
    term = (1.0 / ((double)(k + 1) * (double)(k + 2))) * (term * q);
    psi_k1 += 1.0 / (k + 1);
    psi_k2 += 1.0 / (k + 2);
    if (c_abs(term) < 1e-18 * c_abs(sj)) break;
  }
  *j1 = sj;
  *y1 = c_div(C{-2.0 / kPi, 0.0}, z) + (2.0 / kPi) * (c_log(hx) * sj) - (1.0 / kPi) * sy;
}

}  // namespace lsop_bessel
