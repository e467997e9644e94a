// Voigt function H(a, v) = Re w(v + i a), with w the Faddeeva function, for
// the line profiles of the model atom (Sect. 3.1: Voigt absorption profiles
// with a damping parameter).  Host and device.
//
//   |v| < 8 : Taylor expansion of w about the real axis in the step i a,
//             w(x) = exp(-x^2) + (2 i / sqrt(pi)) D(x), with the derivatives
//             from w' = -2 z w + 2 i / sqrt(pi) and
//             w^(n+1) = -2 z w^(n) - 2 n w^(n-1);
//             Dawson's integral D(x) by Rybicki's exponentially convergent
//             sampling series (G. B. Rybicki 1989, Computers in Physics 3, 85)
//             with step h = 0.25 (aliasing error ~ exp(-(pi/2h)^2) < 1e-17).
//   |v| >= 8: asymptotic expansion w(z) ~ (i / (sqrt(pi) z)) sum_n (2n-1)!! / (2 z^2)^n
//             (Abramowitz & Stegun 7.1.23), 20 terms, plus Re exp(-z^2)
//             which the series omits (it matters only for a -> 0).
// Intended range 0 <= a <= 0.1; relative accuracy ~1e-14.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define NLTE_HD __host__ __device__
#else
#define NLTE_HD
#endif

namespace nlte {

NLTE_HD inline double dawson_rybicki(double x) {
  const double h = 0.25;
  const double n0 = 2.0 * rint(x / (2.0 * h));  // even multiple index
  const double xp = x - n0 * h;                 // |xp| <= h
  const double q = exp(2.0 * xp * h);
  const double q2 = q * q;
  double qp = q, qm = 1.0 / q;
  double sum = 0.0;
  for (int np = 1; np <= 27; np += 2) {
    const double c = exp(-(np * h) * (np * h));
    sum += c * (qp / (np + n0) + qm / (n0 - np));
    qp *= q2;
    qm /= q2;
  }
  return exp(-xp * xp) * sum * 0.56418958354775628695;  // 1/sqrt(pi)
}

NLTE_HD inline double voigt_H(double a, double v) {
  const double x = fabs(v);
  const double inv_sqrt_pi = 0.56418958354775628695;
  if (x >= 8.0) {
    const double zr = x, zi = a;
    const double d = zr * zr + zi * zi;
    const double ur = (zr * zr - zi * zi) / (d * d);
    const double ui = -2.0 * zr * zi / (d * d);
    double c[20];
    c[0] = 1.0;
    for (int n = 1; n < 20; ++n) c[n] = c[n - 1] * (2.0 * n - 1.0) * 0.5;
    double sr = c[19], si = 0.0;
    for (int n = 18; n >= 0; --n) {
      const double tr = sr * ur - si * ui + c[n];
      const double ti = sr * ui + si * ur;
      sr = tr;
      si = ti;
    }
    // plus Re exp(-z^2), the part the asymptotic series omits (matters only
    // when a is ~0)
    return (zi * sr - zr * si) * inv_sqrt_pi / d + exp(-(zr * zr - zi * zi)) * cos(2.0 * zr * zi);
  }
  const double e = exp(-x * x);
  const double two_isp = 2.0 * inv_sqrt_pi;
  // W_n = w^(n)(x), complex; term_n = Re(W_n i^n) a^n / n!
  double w0r = e, w0i = two_isp * dawson_rybicki(x);
  double w1r = -2.0 * x * w0r, w1i = -2.0 * x * w0i + two_isp;
  double H = w0r;
  double fac = a;  // a^n / n!
  double pr = w0r, pi_ = w0i, cr = w1r, ci = w1i;
  double prev = 1.0;
  for (int n = 1; n < 64; ++n) {
    double re;
    switch (n & 3) {
      case 0: re = cr; break;
      case 1: re = -ci; break;
      case 2: re = -cr; break;
      default: re = ci; break;
    }
    const double term = re * fac;
    H += term;
    // even-order terms carry exp(-x^2) and may vanish on their own: stop
    // only after two consecutive negligible terms
    if (n >= 3 && fabs(term) <= 1e-18 * fabs(H) && fabs(prev) <= 1e-18 * fabs(H)) break;
    prev = term;
    // advance: W_{n+1} = -2 x W_n - 2 n W_{n-1}
    const double nr = -2.0 * x * cr - 2.0 * n * pr;
    const double ni = -2.0 * x * ci - 2.0 * n * pi_;
    pr = cr;
    pi_ = ci;
    cr = nr;
    ci = ni;
    fac *= a / (n + 1);
    if (fac == 0.0) break;
  }
  return H;
}

}  // namespace nlte
