// Special functions for the matching coefficients, usable on host and device.
//
// Spherical Bessel functions j_l and their derivatives enter the value and
// slope matching at the muffin-tin radius; the complex spherical harmonics
// enter the angular factor of the coefficients (Eq. 2).
#pragma once

#include <hip/hip_runtime.h>

namespace hsb {

constexpr int kMaxL = 12;  // largest l_max; j_l is needed up to l_max + 1

// j_0..j_nmax at x >= 0 into j[].
//  * x < 2: the power series j_l(x) = x^l/(2l+1)!! sum_k (-x^2/2)^k / (k! prod_{i=1..k}(2l+2i+1)),
//    whose terms shrink fast and alternate with little cancellation there;
//  * x >= 2: Miller's backward recurrence f_{n-1} = (2n+1)/x f_n - f_{n+1}
//    from an index well above both nmax and x, scaled to the closed forms of
//    j_0 and j_1 by least squares (robust at the zeros of either).
__host__ __device__ inline void sph_bessel_seq(int nmax, double x, double* j) {
  if (x < 2.0) {
    const double y = -0.5 * x * x;
    double pref = 1.0;  // x^l / (2l+1)!!
    for (int l = 0; l <= nmax; ++l) {
      if (l > 0) pref *= x / (2.0 * l + 1.0);
      double t = 1.0, s = 1.0;
      for (int k = 1; k < 40; ++k) {
        t *= y / (k * (2.0 * l + 2.0 * k + 1.0));
        s += t;
        if (fabs(t) < 1e-18 * fabs(s)) break;
      }
      j[l] = pref * s;
    }
    return;
  }
  // requires nmax >= 1 (j_0 and j_1 fix the scale)
  const double inv = 1.0 / x;
  const int start = nmax + 24 + (int)x;
  double fp1 = 0.0, f = 1.0;
  for (int n = start; n >= 1; --n) {
    const double fm1 = (2.0 * n + 1.0) * inv * f - fp1;
    fp1 = f;
    f = fm1;
    const int idx = n - 1;  // f holds f_{n-1}, fp1 holds f_n
    if (idx <= nmax) j[idx] = f;
    if (idx + 1 <= nmax) j[idx + 1] = fp1;
    if (fabs(f) > 1e250) {  // rescale to stay finite
      f *= 1e-250;
      fp1 *= 1e-250;
      for (int m = idx; m <= nmax; ++m) j[m] *= 1e-250;
    }
  }
  // least-squares scale on (f_0, f_1), normalised first so the squares cannot underflow
  const double fm = fmax(fabs(j[0]), fabs(j[1]));
  const double f0 = j[0] / fm, f1 = j[1] / fm;
  double s, c;
  sincos(x, &s, &c);
  const double j0 = s * inv, j1 = (s * inv - c) * inv;
  const double scale = (j0 * f0 + j1 * f1) / ((f0 * f0 + f1 * f1) * fm);
  for (int l = 0; l <= nmax; ++l) j[l] *= scale;
}

// j_l'(x) for l = 0..lmax from j_0..j_{lmax+1}:  j_0' = -j_1,
// j_l' = (l j_{l-1} - (l+1) j_{l+1}) / (2l+1).
__host__ __device__ inline void sph_bessel_deriv(int lmax, const double* j, double* dj) {
  dj[0] = -j[1];
  for (int l = 1; l <= lmax; ++l) dj[l] = (l * j[l - 1] - (l + 1) * j[l + 1]) / (2.0 * l + 1.0);
}

// Visits pre * i^l * conj(Y_lm(K_hat)) for every (l, m) in L order
// (L = l^2 + l + m), calling emit(L, re, im).  Y_lm = Pbar_lm(cos t) (sin t e^{i phi})^m
// for m >= 0 with the fully normalised Legendre factor Pbar carrying the
// Condon-Shortley sign, and Y_{l,-m} = (-1)^m conj(Y_lm).  The powers of
// sin t e^{i phi} = (Kx + i Ky)/|K| avoid explicit angles.
template <class Emit>
__host__ __device__ inline void angular_visit(int lmax, double kx, double ky, double kz, double pre, Emit emit) {
  const double kn = sqrt(kx * kx + ky * ky + kz * kz);
  double ct, wr, wi;  // cos(theta), (sin theta e^{i phi}) = wr + i wi
  if (kn < 1e-12) {
    ct = 1.0; wr = 0.0; wi = 0.0;
  } else {
    const double r = 1.0 / kn;
    ct = kz * r; wr = kx * r; wi = ky * r;
  }
  // pmm = Pbar_mm without its sin^m factor; wm = w^m
  double pmm = 0.28209479177387814347;  // 1/sqrt(4 pi)
  double wmr = 1.0, wmi = 0.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) {
      pmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m));
      const double tr = wmr * wr - wmi * wi, ti = wmr * wi + wmi * wr;
      wmr = tr; wmi = ti;
    }
    double p_lm2 = 0.0, p_lm1 = 0.0;
    for (int l = m; l <= lmax; ++l) {
      double p;
      if (l == m) {
        p = pmm;
      } else if (l == m + 1) {
        p = sqrt(2.0 * m + 3.0) * ct * pmm;
      } else {
        const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double b = sqrt((((double)(l - 1) * (l - 1)) - (double)m * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
        p = a * (ct * p_lm1 - b * p_lm2);
      }
      p_lm2 = p_lm1;
      p_lm1 = p;
      // Y_lm = p * w^m ; conj(Y_lm) = p * conj(w^m)
      const double yr = p * wmr, yi = -p * wmi;  // conj(Y_lm)
      // i^l
      double cr, ci;
      switch (l & 3) {
        case 0: cr = yr; ci = yi; break;
        case 1: cr = -yi; ci = yr; break;
        case 2: cr = -yr; ci = -yi; break;
        default: cr = yi; ci = -yr; break;
      }
      emit(l * l + l + m, pre * cr, pre * ci);
      if (m > 0) {
        // conj(Y_{l,-m}) = (-1)^m Y_lm = (-1)^m p w^m
        const double sg = (m & 1) ? -1.0 : 1.0;
        const double nr = sg * p * wmr, ni = sg * p * wmi;
        switch (l & 3) {
          case 0: cr = nr; ci = ni; break;
          case 1: cr = -ni; ci = nr; break;
          case 2: cr = -nr; ci = -ni; break;
          default: cr = ni; ci = -nr; break;
        }
        emit(l * l + l - m, pre * cr, pre * ci);
      }
    }
  }
}

}  // namespace hsb
