// Device kernel functions shared by the dense assembly and the accelerator's
// near-field assembly: the double-layer kernel of the shifted Green function
// and one matrix entry of the direct operator for a given source image.
#pragma once
#include "sesm_impl.h"

// K_dl per unit dx' (upward normal (-f', 1) dx' = nu ds'):
//   sum_m (-1)^m C(j,m) (ik/4) H1(k R_m) (Y + m h - f'(x') X) / R_m,
// X = x - x', Y = f(x) - f(x'), R_m = |(X, Y + m h)|  (eqs. shifted_green_function, K_def).
__device__ inline cplx sesm_kdl(const KParams& K, double X, double Y, double fps) {
  cplx acc = cplx{0.0, 0.0};
  for (int m = 0; m <= K.j; ++m) {
    const double Ym = Y + m * K.h;
    const double R = sqrt(X * X + Ym * Ym);
    const cplx H1 = sesm_hankel1(K.k * R);
    acc += (K.wshift[m] * (Ym - fps * X) / R) * H1;
  }
  return (0.25 * K.k) * mul_i(acc);
}

// Regular + singular contribution of one source image (X != 0 or Y != 0):
//   dx (1 - S^f) K_dl + S^f (R_m K_s + dx K_r),  K_r = K_dl - K_s ln(4 sin^2(pi X/a))
// (eqs. DAdx_def and local_mat; K_s the Martensen-Kussmaul coefficient of eq. ks_def).
// SA multiplies the regular part (window S_{cA,A}; equal to 1 for near images).
__device__ inline cplx sesm_entry_offdiag(const KParams& K, const double* __restrict__ logw, double X, double Y,
                                          double fps, double SA) {
  const double r = sqrt(X * X + Y * Y);
  const double Sf = sesm_window(r, K.gamma, K.a);
  const cplx Kd = sesm_kdl(K, X, Y, fps);
  cplx term = (K.dx * SA * (1.0 - Sf)) * Kd;
  if (Sf > 0.0) {
    const double Ks = (K.k / (4.0 * SESM_PI)) * (fps * X - Y) * sesm_besselj1(K.k * r) / r;
    const double sn = sin(SESM_PI * X / K.a);
    const double lg = log(4.0 * sn * sn);
    int m = (int)llrint(-X / K.dx);
    m = m < 0 ? -m : m;
    m %= K.n_a;
    term += Sf * (cplx{logw[m] * Ks, 0.0} + K.dx * (Kd - cplx{Ks * lg, 0.0}));
  }
  return term;
}

// Diagonal: D~_sing contributes dx K_r(x,x) (K_s(x,x) = 0), plus 1/2:
//   K_r(x,x) = f''/(4 pi (1 + f'^2)) + sum_{m>=1} (-1)^m C(j,m) (ik/4) H1(k m h).
__device__ inline cplx sesm_entry_diag(const KParams& K, double fp, double fpp) {
  cplx kr = cplx{fpp / (4.0 * SESM_PI * (1.0 + fp * fp)), 0.0};
  for (int m = 1; m <= K.j; ++m) kr += (0.25 * K.k * K.wshift[m]) * mul_i(sesm_hankel1(K.k * m * K.h));
  cplx out = K.dx * kr;
  out.re += 0.5;
  return out;
}
