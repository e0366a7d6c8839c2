// Adjoint gradients of efficiency objectives with respect to the profile's
// Fourier coefficients (dense mode).
//
// The discrete problem is (1/2 I + D^dx(f)) mu = b(f) (eq. discrete_eq); an
// objective J = sum_n w_n e_n over the propagating orders, with
// e_n = (beta_n / beta) |B_n|^2 and B_n = sum_l c_n(l) mu_l the Rayleigh
// coefficients of the solution, depends on the profile f through c_n, b and
// the operator.  With a_n = w_n (beta_n / beta) conj(B_n) and
// g_l = sum_n a_n c_n(l), the adjoint density nu solves
// (1/2 I + D^dx)^H nu = conj(g), and for a perturbation theta of the profile
//   dJ/dtheta = 2 Re[ sum_n a_n sum_l (dc_n(l)/dtheta) mu_l
//                     + sum_i conj(nu_i) (db_i/dtheta - sum_l (dA_il/dtheta) mu_l) ].
// Every entry A_il depends on the profile through Y = f(x_i) - f(x_l) and
// the source slope f'(x_l) (the double-layer kernel, eqs. K_def and
// shifted_green_function; the singular split of eq. local_mat through the 2-D
// distance of its window and K_s of eq. ks_def; the completion modes through
// beta_n Y and J_l), the diagonal also through f'(x_i) and f''(x_i)
// (K_r(x, x)).  The derivative matrices DY = dA/dY and DF = dA/df'_l are
// assembled like the operator itself, so that
//   sum_il conj(nu_i) (dA_il/dtheta) mu_l = sum_k [ (conj(nu_k) (DY mu)_k - mu_k (DY^T conj(nu))_k) phi(x_k)
//                                                  + mu_k (DF^T conj(nu))_k phi'(x_k)
//                                                  + conj(nu_k) mu_k dA_kk/df''_k phi''(x_k) ],
// phi the perturbation of f (cos / sin of the Fourier mode).
#include <cmath>
#include <vector>

#include "sesm.h"
#include "sesm_kernels.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

// d/dx of the window S_{gamma,a}(x) of eq. (S_def), for x >= 0
__device__ inline double window_dx(double x, double gamma, double a) {
  if (x <= gamma || x >= a) return 0.0;
  const double u = (x - gamma) / (a - gamma);
  const double e = exp(-1.0 / u);
  const double g = 2.0 * e / (u - 1.0);
  const double dg = 2.0 * e * ((u - 1.0) / (u * u) - 1.0) / ((u - 1.0) * (u - 1.0));
  return exp(g) * dg / (a - gamma);
}

// dK_dl/dY and dK_dl/df' of the shifted double-layer kernel (K_dl of sesm_kdl):
//   d/dY [H1(kR) (Y_m - f'X)/R] = H1/R + (Y_m - f'X) (Y_m/R) (k H0(kR)/R - 2 H1(kR)/R^2),
//   d/df' [H1(kR) (Y_m - f'X)/R] = -X H1(kR)/R.
__device__ inline void kdl_deriv(const KParams& K, double X, double Y, double fps, cplx* dY, cplx* dF) {
  cplx ay = cplx{0.0, 0.0}, af = cplx{0.0, 0.0};
  for (int m = 0; m <= K.j; ++m) {
    const double Ym = Y + m * K.h;
    const double R = sqrt(X * X + Ym * Ym);
    cplx H0, H1;
    sesm_hankel01(K.k * R, &H0, &H1);
    const double num = Ym - fps * X;
    const cplx dR = (K.k / R) * H0 - (2.0 / (R * R)) * H1;  // d/dR (H1(kR)/R)
    ay += K.wshift[m] * ((1.0 / R) * H1 + (num * Ym / R) * dR);
    af += (-K.wshift[m] * X / R) * H1;
  }
  *dY = (0.25 * K.k) * mul_i(ay);
  *dF = (0.25 * K.k) * mul_i(af);
}

// Derivatives of sesm_entry_offdiag (one source image) in Y and f'_l:
//   entry = dx SA (1 - Sf) Kd + Sf (R_m Ks + dx (Kd - Ks lg)),  Sf = S_{gamma,a}(r), r = |(X, Y)|,
//   Ks = (k/4pi) (f' X - Y) J1(kr)/r,  d/dr (J1(kr)/r) = k J0(kr)/r - 2 J1(kr)/r^2.
__device__ inline void entry_offdiag_deriv(const KParams& K, const double* __restrict__ logw, double X, double Y,
                                           double fps, double SA, cplx* dY, cplx* dF) {
  const double r = sqrt(X * X + Y * Y);
  const double Sf = sesm_window(r, K.gamma, K.a);
  cplx dKy, dKf;
  kdl_deriv(K, X, Y, fps, &dKy, &dKf);
  cplx ey = (K.dx * SA * (1.0 - Sf)) * dKy, ef = (K.dx * SA * (1.0 - Sf)) * dKf;
  const double dSf = window_dx(r, K.gamma, K.a) * (r > 0.0 ? Y / r : 0.0);
  if (Sf > 0.0 || dSf != 0.0) {
    const cplx Kd = sesm_kdl(K, X, Y, fps);
    cplx H0, H1;
    sesm_hankel01(K.k * r, &H0, &H1);
    const double J0 = H0.re, J1 = H1.re;
    const double c = K.k / (4.0 * SESM_PI);
    const double Ks = c * (fps * X - Y) * J1 / r;
    const double dJr = K.k * J0 / r - 2.0 * J1 / (r * r);
    const double dKs_y = c * (-J1 / r + (fps * X - Y) * dJr * (Y / r));
    const double dKs_f = c * X * J1 / r;
    const double sn = sin(SESM_PI * X / K.a);
    const double lg = log(4.0 * sn * sn);
    int m = (int)llrint(-X / K.dx);
    m = m < 0 ? -m : m;
    m %= K.n_a;
    const double Rm = logw[m];
    // window terms
    ey += dSf * (cplx{Rm * Ks, 0.0} + K.dx * (Kd - cplx{Ks * lg, 0.0}) - (K.dx * SA) * Kd);
    ey += Sf * (cplx{Rm * dKs_y, 0.0} + K.dx * (dKy - cplx{dKs_y * lg, 0.0}));
    ef += Sf * (cplx{Rm * dKs_f, 0.0} + K.dx * (dKf - cplx{dKs_f * lg, 0.0}));
  }
  *dY = ey;
  *dF = ef;
}

// One source image: the entry of sesm_entry_offdiag and its two derivatives
// of entry_offdiag_deriv in one evaluation, the Hankel functions of each
// shifted image computed once (H1 for the entry, H0 and H1 for the
// derivatives; the entry's own terms in the same order as sesm_entry_offdiag).
__device__ inline void entry_and_derivs(const KParams& K, const double* __restrict__ logw, double X, double Y,
                                        double fps, double SA, cplx* ent, cplx* dY, cplx* dF) {
  cplx kd = cplx{0.0, 0.0}, ay = cplx{0.0, 0.0}, af = cplx{0.0, 0.0};
  for (int m = 0; m <= K.j; ++m) {
    const double Ym = Y + m * K.h;
    const double R = sqrt(X * X + Ym * Ym);
    cplx H0, H1;
    sesm_hankel01(K.k * R, &H0, &H1);
    kd += (K.wshift[m] * (Ym - fps * X) / R) * H1;
    const double num = Ym - fps * X;
    const cplx dR = (K.k / R) * H0 - (2.0 / (R * R)) * H1;  // d/dR (H1(kR)/R)
    ay += K.wshift[m] * ((1.0 / R) * H1 + (num * Ym / R) * dR);
    af += (-K.wshift[m] * X / R) * H1;
  }
  const cplx Kd = (0.25 * K.k) * mul_i(kd);
  const cplx dKy = (0.25 * K.k) * mul_i(ay), dKf = (0.25 * K.k) * mul_i(af);
  const double r = sqrt(X * X + Y * Y);
  const double Sf = sesm_window(r, K.gamma, K.a);
  cplx term = (K.dx * SA * (1.0 - Sf)) * Kd;
  cplx ey = (K.dx * SA * (1.0 - Sf)) * dKy, ef = (K.dx * SA * (1.0 - Sf)) * dKf;
  const double dSf = window_dx(r, K.gamma, K.a) * (r > 0.0 ? Y / r : 0.0);
  if (Sf > 0.0 || dSf != 0.0) {
    const double sn = sin(SESM_PI * X / K.a);
    const double lg = log(4.0 * sn * sn);
    int mi = (int)llrint(-X / K.dx);
    mi = mi < 0 ? -mi : mi;
    mi %= K.n_a;
    const double Rm = logw[mi];
    if (Sf > 0.0) {
      const double Ks = (K.k / (4.0 * SESM_PI)) * (fps * X - Y) * sesm_besselj1(K.k * r) / r;
      term += Sf * (cplx{Rm * Ks, 0.0} + K.dx * (Kd - cplx{Ks * lg, 0.0}));
    }
    cplx H0, H1;
    sesm_hankel01(K.k * r, &H0, &H1);
    const double J0 = H0.re, J1 = H1.re;
    const double c = K.k / (4.0 * SESM_PI);
    const double Ks = c * (fps * X - Y) * J1 / r;
    const double dJr = K.k * J0 / r - 2.0 * J1 / (r * r);
    const double dKs_y = c * (-J1 / r + (fps * X - Y) * dJr * (Y / r));
    const double dKs_f = c * X * J1 / r;
    ey += dSf * (cplx{Rm * Ks, 0.0} + K.dx * (Kd - cplx{Ks * lg, 0.0}) - (K.dx * SA) * Kd);
    ey += Sf * (cplx{Rm * dKs_y, 0.0} + K.dx * (dKy - cplx{dKs_y * lg, 0.0}));
    ef += Sf * (cplx{Rm * dKs_f, 0.0} + K.dx * (dKf - cplx{dKs_f * lg, 0.0}));
  }
  *ent = term;
  *dY = ey;
  *dF = ef;
}

// The dense operator (as k_dense_assemble) together with DY and DF (as
// k_dense_deriv), one wave per entry, lanes over the source images.
__global__ __launch_bounds__(256) void k_dense_assemble_deriv(KParams K, const double* __restrict__ x,
                                                              const double* __restrict__ f,
                                                              const double* __restrict__ fp,
                                                              const double* __restrict__ fpp,
                                                              const double* __restrict__ J,
                                                              const double* __restrict__ logw, cplx* __restrict__ M,
                                                              cplx* __restrict__ DY, cplx* __restrict__ DF) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y;
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= K.N) return;  // wave-uniform
  const int64_t e = (int64_t)i * K.N + l;
  const double X0 = x[i] - x[l], Y = f[i] - f[l], fps = fp[l];
  cplx acc = cplx{0.0, 0.0}, ay = cplx{0.0, 0.0}, af = cplx{0.0, 0.0};
  for (int p = K.pmin + lane; p <= K.pmax; p += 64) {
    const double Xp = X0 - p * K.d;
    const double SA = sesm_window(Xp, K.cA, K.A_len);
    if (SA == 0.0) continue;
    if (p == 0 && i == l) continue;  // diagonal: handled below
    cplx en, dy, df;
    entry_and_derivs(K, logw, Xp, Y, fps, SA, &en, &dy, &df);
    const cplx ph = cexp_i(K.alpha * p * K.d);
    acc += ph * en;
    ay += ph * dy;
    af += ph * df;
  }
  acc = wave_sum(acc);
  ay = wave_sum(ay);
  af = wave_sum(af);
  if (lane == 0) {
    if (i == l) {
      acc += sesm_entry_diag(K, fp[i], fpp[i]);
      const double q = 1.0 + fps * fps;
      af.re += K.dx * (-fpp[i] * fps / (2.0 * SESM_PI * q * q));
    }
    for (int t = 0; t < K.nU; ++t) {
      const double mag = exp(-K.Ubi[t] * Y);
      acc += (mag * J[l] * K.dx) * cexp_i(K.Ua[t] * X0 + K.Ubr[t] * Y);
      const cplx e0 = (exp(-K.Ubi[t] * Y) * K.dx) * cexp_i(K.Ua[t] * X0 + K.Ubr[t] * Y);
      ay += (J[l] * e0) * cplx{-K.Ubi[t], K.Ubr[t]};  // i beta_n
      af += (fps / J[l]) * e0;
    }
    M[e] = acc;
    DY[e] = ay;
    DF[e] = af;
  }
}

// DY[i][l] = dA_il/dY, DF[i][l] = dA_il/df'_l (the diagonal: df'_i, with the
// K_r(x, x) term), over the images p as in the assembly; one wave per entry.
__global__ __launch_bounds__(256) void k_dense_deriv(KParams K, const double* __restrict__ x,
                                                     const double* __restrict__ f, const double* __restrict__ fp,
                                                     const double* __restrict__ fpp, const double* __restrict__ J,
                                                     const double* __restrict__ logw, cplx* __restrict__ DY,
                                                     cplx* __restrict__ DF) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y;
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= K.N) return;  // wave-uniform
  const int64_t e = (int64_t)i * K.N + l;
  const double X0 = x[i] - x[l], Y = f[i] - f[l], fps = fp[l];
  cplx ay = cplx{0.0, 0.0}, af = cplx{0.0, 0.0};
  for (int p = K.pmin + lane; p <= K.pmax; p += 64) {
    const double Xp = X0 - p * K.d;
    const double SA = sesm_window(Xp, K.cA, K.A_len);
    if (SA == 0.0) continue;
    if (p == 0 && i == l) continue;
    cplx dy, df;
    entry_offdiag_deriv(K, logw, Xp, Y, fps, SA, &dy, &df);
    const cplx ph = cexp_i(K.alpha * p * K.d);
    ay += ph * dy;
    af += ph * df;
  }
  ay = wave_sum(ay);
  af = wave_sum(af);
  if (lane == 0) {
    if (i == l) {  // K_r(x, x) = f'' / (4 pi (1 + f'^2)) + ...: d/df'
      const double q = 1.0 + fps * fps;
      af.re += K.dx * (-fpp[i] * fps / (2.0 * SESM_PI * q * q));
    }
    for (int t = 0; t < K.nU; ++t) {  // completion modes J_l dx e^{i alpha_n X + i beta_n Y}
      const cplx e0 = (exp(-K.Ubi[t] * Y) * K.dx) * cexp_i(K.Ua[t] * X0 + K.Ubr[t] * Y);
      ay += (J[l] * e0) * cplx{-K.Ubi[t], K.Ubr[t]};  // i beta_n
      af += (fps / J[l]) * e0;
    }
    DY[e] = ay;
    DF[e] = af;
  }
}

// y = M^H x (CONJ; M^T x otherwise): 64 columns per workgroup (lane =
// column; each wavefront load reads 1 KB of a row), the sixteen wavefronts
// take every sixteenth row with eight rows' loads in flight per lane, and
// their partial sums are added in LDS in a fixed order.  (With N / 64
// workgroups the launch is narrow, hence the many rows in flight per
// workgroup.)
template <bool CONJ>
__global__ __launch_bounds__(1024) void k_gemv_cols(int N, const cplx* __restrict__ M, const cplx* __restrict__ x,
                                                    cplx* __restrict__ y) {
  constexpr int NW = 16, U = 8;
  __shared__ cplx part[NW][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l = blockIdx.x * 64 + lane;
  const int lc = min(l, N - 1);  // lanes past N repeat the last column (not stored)
  cplx acc = cplx{0.0, 0.0};
  int i = wv;
  for (; i + NW * (U - 1) < N; i += NW * U) {
    cplx m[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      m[u] = load_stream(&M[(int64_t)(i + NW * u) * N + lc]);
      xv[u] = x[i + NW * u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = cmac(acc, CONJ ? conj(m[u]) : m[u], xv[u]);
  }
  for (; i < N; i += NW) {
    const cplx m = load_stream(&M[(int64_t)i * N + lc]);
    acc = cmac(acc, CONJ ? conj(m) : m, x[i]);
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && l < N) {
    cplx sm = part[0][lane];
    for (int w = 1; w < NW; ++w) sm += part[w][lane];
    y[l] = sm;
  }
}

// y = M x, one workgroup per row
__global__ __launch_bounds__(256) void k_gemv_rows_g(int N, const cplx* __restrict__ M, const cplx* __restrict__ x,
                                                     cplx* __restrict__ y) {
  __shared__ cplx sh[4];
  const cplx* row = M + (int64_t)blockIdx.x * N;
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < N; l += 256) acc += load_stream(&row[l]) * x[l];
  const cplx s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) y[blockIdx.x] = s;
}

// The order records of the objective: alpha_n, beta_n (real, propagating),
// Q_n = (1 - e^{i beta_n h})^j / beta_n (its beta_n -> 0 limit at a Wood
// anomaly), membership in U^eta, weight.
struct Order {
  double an, bn;
  cplx Q;
  int inU;
  double w;
};

__device__ inline cplx coef_c(const KParams& K, const Order& o, double xl, double fl, double fpl, double Jl) {
  // c_n(l) = dx [-(alpha_n f'_l - beta_n) Q_n / (2d) + 1[n in U] J_l] e^{-i alpha_n x_l - i beta_n f_l}
  cplx v = (-(o.an * fpl - o.bn) / (2.0 * K.d)) * o.Q;
  if (o.inU) v.re += Jl;
  return K.dx * v * cexp_i(-o.an * xl - o.bn * fl);
}
__device__ inline cplx coef_c_dfp(const KParams& K, const Order& o, double xl, double fl, double fpl, double Jl) {
  cplx v = (-o.an / (2.0 * K.d)) * o.Q;
  if (o.inU) v.re += fpl / Jl;
  return K.dx * v * cexp_i(-o.an * xl - o.bn * fl);
}

// B_n = sum_l c_n(l) mu_l, one workgroup per order
__global__ __launch_bounds__(256) void k_grad_B(KParams K, const Order* __restrict__ ord,
                                                const double* __restrict__ x, const double* __restrict__ f,
                                                const double* __restrict__ fp, const double* __restrict__ J,
                                                const cplx* __restrict__ mu, cplx* __restrict__ B) {
  __shared__ cplx sh[4];
  const Order o = ord[blockIdx.x];
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < K.N; l += 256) acc += coef_c(K, o, x[l], f[l], fp[l], J[l]) * mu[l];
  const cplx s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) B[blockIdx.x] = s;
}

// adjoint right-hand side conj(g_l), g_l = sum_n a_n c_n(l); one thread per node
__global__ void k_grad_rhs(KParams K, int no, const Order* __restrict__ ord, const cplx* __restrict__ a,
                           const double* __restrict__ x, const double* __restrict__ f, const double* __restrict__ fp,
                           const double* __restrict__ J, cplx* __restrict__ rhs) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K.N) return;
  cplx g = cplx{0.0, 0.0};
  for (int t = 0; t < no; ++t) g += a[t] * coef_c(K, ord[t], x[l], f[l], fp[l], J[l]);
  rhs[l] = conj(g);
}

// per node: the coefficients of phi, phi', phi'' in dJ/dtheta / 2 (real part taken later)
__global__ void k_grad_nodes(KParams K, int no, const Order* __restrict__ ord, const cplx* __restrict__ a,
                             double beta, const double* __restrict__ x, const double* __restrict__ f,
                             const double* __restrict__ fp, const double* __restrict__ fpp,
                             const double* __restrict__ J, const cplx* __restrict__ mu, const cplx* __restrict__ nu,
                             const cplx* __restrict__ DYmu, const cplx* __restrict__ DYtnu,
                             const cplx* __restrict__ DFtnu, cplx* __restrict__ Pk, cplx* __restrict__ Qk,
                             cplx* __restrict__ Rk) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K.N) return;
  cplx sc = cplx{0.0, 0.0}, sf = cplx{0.0, 0.0};
  for (int t = 0; t < no; ++t) {
    const Order& o = ord[t];
    sc += a[t] * (o.bn * mul_i(-1.0 * coef_c(K, o, x[k], f[k], fp[k], J[k])));  // dc/df = -i beta_n c
    sf += a[t] * coef_c_dfp(K, o, x[k], f[k], fp[k], J[k]);
  }
  const cplx m = mu[k], cn = conj(nu[k]);
  // b_k = -e^{i (alpha x_k - beta f_k)}, db_k/df_k = i beta e^{i (alpha x_k - beta f_k)}
  const cplx db = beta * mul_i(cexp_i(K.alpha * x[k] - beta * f[k]));
  Pk[k] = sc * m + cn * db - (cn * DYmu[k] - m * DYtnu[k]);
  Qk[k] = sf * m - m * DFtnu[k];
  const double q = 1.0 + fp[k] * fp[k];
  Rk[k] = (-K.dx / (4.0 * SESM_PI * q)) * (cn * m);
}

// dJ/da_m, dJ/db_m = 2 Re sum_k [P_k phi + Q_k phi' + R_k phi''] with
// phi = cos(2 pi m x/d) (a_m) or sin(2 pi m x/d) (b_m); one workgroup per (m, kind)
__global__ __launch_bounds__(256) void k_grad_modes(int N, double d, const double* __restrict__ x,
                                                    const cplx* __restrict__ Pk, const cplx* __restrict__ Qk,
                                                    const cplx* __restrict__ Rk, double* __restrict__ ga,
                                                    double* __restrict__ gb) {
  __shared__ cplx sh[4];
  const int m = blockIdx.x >> 1, kind = blockIdx.x & 1;
  const double km = 2.0 * kPi * m / d;
  cplx acc = cplx{0.0, 0.0};
  for (int k = threadIdx.x; k < N; k += 256) {
    double s, c;
    sincos(km * x[k], &s, &c);
    const double ph = kind == 0 ? c : s, dph = kind == 0 ? -km * s : km * c, d2 = -km * km * ph;
    acc += ph * Pk[k] + dph * Qk[k] + d2 * Rk[k];
  }
  const cplx t = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) {
    if (kind == 0) ga[m] = 2.0 * t.re;
    else gb[m] = m == 0 ? 0.0 : 2.0 * t.re;
  }
}

// the propagating orders with their weights (host)
int build_orders(sesm_ctx* ctx, const double* w, int n_w, std::vector<Order>& ord) {
  const Problem& P = ctx->P;
  if (n_w != P.n_count) return ctx->fail(SESM_EINVAL, "objective: need one weight per propagating order (n_count)");
  ord.clear();
  for (int t = 0; t < P.n_count; ++t) {
    if (!std::isfinite(w[t])) return ctx->fail(SESM_EINVAL, "objective: non-finite weight");
    const int n = P.n_first + t;
    Order o;
    o.an = P.alpha + 2.0 * kPi * n / P.d;
    const double g = (P.k - o.an) * (P.k + o.an);
    o.bn = g > 0.0 ? std::sqrt(g) : 0.0;
    // (1 - e^{i beta h})^j / beta = (-2i)^j sin^{j-1}(beta h/2) (h/2) sinc(beta h/2) e^{i j beta h/2}
    const double z = 0.5 * P.h * o.bn;
    const double sz = std::sin(z), sinc = std::fabs(z) < 1e-8 ? 1.0 - z * z / 6.0 : std::sin(z) / z;
    double mag = 0.5 * P.h * sinc;
    for (int m = 1; m < P.j; ++m) mag *= sz;
    cplx c2 = cplx{1.0, 0.0};
    for (int m = 0; m < P.j; ++m) c2 = cplx{2.0 * c2.im, -2.0 * c2.re};
    const double ph = P.j * z;
    o.Q = cplx{mag * (c2.re * std::cos(ph) - c2.im * std::sin(ph)), mag * (c2.re * std::sin(ph) + c2.im * std::cos(ph))};
    if (P.j == 0) o.Q = o.bn > 0.0 ? cplx{1.0 / o.bn, 0.0} : cplx{0.0, 0.0};
    o.inU = 0;
    for (int u = 0; u < P.nU; ++u) o.inU |= P.U[u] == n;
    o.w = w[t];
    ord.push_back(o);
  }
  return SESM_OK;
}

// a_n = w_n (beta_n / beta) conj(B_n) on the host, after B_n on the device
int objective_weights(sesm_ctx* ctx, const cplx* mu, const std::vector<Order>& ord, Order* dord, cplx* dB,
                      std::vector<cplx>& a, double* J) {
  const Problem& P = ctx->P;
  const KParams K = ctx->kparams();
  const int no = (int)ord.size();
  SESM_HIP(hipMemcpyAsync(dord, ord.data(), sizeof(Order) * no, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_grad_B, dim3(no), dim3(256), 0, ctx->stream, K, dord, ctx->x, ctx->f, ctx->fp, ctx->J, mu, dB);
  SESM_LAUNCH_CHECK();
  std::vector<cplx> B(no);
  SESM_HIP(hipMemcpyAsync(B.data(), dB, sizeof(cplx) * no, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  a.resize(no);
  double Jv = 0.0;
  for (int t = 0; t < no; ++t) {
    const double s = ord[t].w * ord[t].bn / P.beta;
    Jv += s * (B[t].re * B[t].re + B[t].im * B[t].im);
    a[t] = cplx{s * B[t].re, -s * B[t].im};
  }
  if (J) *J = Jv;
  return SESM_OK;
}

}  // namespace

extern "C" int sesm_objective_adjoint_rhs(sesm_ctx* ctx, const sesm_c64* mu, const double* w, int32_t n_w,
                                          sesm_c64* rhs, double* J) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu || !w || !rhs) return ctx->fail(SESM_EINVAL, "null pointer");
  SESM_HIP(hipSetDevice(ctx->device));
  std::vector<Order> ord;
  int rc = build_orders(ctx, w, n_w, ord);
  if (rc) return rc;
  const int no = (int)ord.size();
  char* buf = nullptr;
  SESM_HIP(hipMalloc((void**)&buf, (sizeof(Order) + 2 * sizeof(cplx)) * (size_t)std::max(no, 1) + 256));
  Order* dord = (Order*)buf;
  cplx* dB = (cplx*)(buf + ((sizeof(Order) * (size_t)std::max(no, 1) + 15) / 16 * 16));
  cplx* da = dB + std::max(no, 1);
  std::vector<cplx> a;
  rc = objective_weights(ctx, (const cplx*)mu, ord, dord, dB, a, J);
  if (rc == SESM_OK) {
    const KParams K = ctx->kparams();
    (void)hipMemcpyAsync(da, a.data(), sizeof(cplx) * no, hipMemcpyHostToDevice, ctx->stream);
    hipLaunchKernelGGL(k_grad_rhs, dim3((ctx->P.N + 255) / 256), dim3(256), 0, ctx->stream, K, no, dord, da, ctx->x,
                       ctx->f, ctx->fp, ctx->J, (cplx*)rhs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(e));
  }
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (rc == SESM_OK && es != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(es));
  return rc;
}

extern "C" int sesm_shape_gradient(sesm_ctx* ctx, const sesm_c64* mu_, const sesm_c64* nu_, const double* w,
                                   int32_t n_w, int32_t n_modes, double* grad_a, double* grad_b) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_DENSE) return ctx->fail(SESM_EINVAL, "shape gradients need the dense mode");
  if (!mu_ || !nu_ || !w || !grad_a || !grad_b) return ctx->fail(SESM_EINVAL, "null pointer");
  if (n_modes < 0 || n_modes > (1 << 20)) return ctx->fail(SESM_EINVAL, "n_modes must be in [0, 2^20]");
  SESM_HIP(hipSetDevice(ctx->device));
  const Problem& P = ctx->P;
  const int N = P.N;
  std::vector<Order> ord;
  int rc = build_orders(ctx, w, n_w, ord);
  if (rc) return rc;
  const int no = (int)ord.size(), nob = std::max(no, 1);
  const cplx* mu = (const cplx*)mu_;
  const cplx* nu = (const cplx*)nu_;
  // work space: DY, DF (N x N each, unless the set-up kept them), conj(nu),
  // three contractions, P, Q, R, orders, B, a, gradients
  const bool kept = ctx->dA_dY && ctx->dA_dF;
  const size_t NN = kept ? 0 : (size_t)N * N;
  const size_t bytes = sizeof(cplx) * (2 * NN + 7 * (size_t)N + 2 * (size_t)nob) + sizeof(Order) * nob +
                       sizeof(double) * 2 * ((size_t)n_modes + 1) + 16 * 256;  // (each piece rounded up to 256 B)
  char* buf = nullptr;
  SESM_HIP(hipMalloc((void**)&buf, bytes));
  char* cur = buf;
  auto take = [&](size_t b) {
    char* p = cur;
    cur += (b + 255) / 256 * 256;
    return (void*)p;
  };
  cplx* DY = kept ? ctx->dA_dY : (cplx*)take(sizeof(cplx) * NN);
  cplx* DF = kept ? ctx->dA_dF : (cplx*)take(sizeof(cplx) * NN);
  cplx* cnu = (cplx*)take(sizeof(cplx) * N);
  cplx* DYmu = (cplx*)take(sizeof(cplx) * N);
  cplx* DYtnu = (cplx*)take(sizeof(cplx) * N);
  cplx* DFtnu = (cplx*)take(sizeof(cplx) * N);
  cplx* Pk = (cplx*)take(sizeof(cplx) * N);
  cplx* Qk = (cplx*)take(sizeof(cplx) * N);
  cplx* Rk = (cplx*)take(sizeof(cplx) * N);
  Order* dord = (Order*)take(sizeof(Order) * nob);
  cplx* dB = (cplx*)take(sizeof(cplx) * nob);
  cplx* da = (cplx*)take(sizeof(cplx) * nob);
  double* dga = (double*)take(sizeof(double) * ((size_t)n_modes + 1));
  double* dgb = (double*)take(sizeof(double) * ((size_t)n_modes + 1));
  std::vector<cplx> a, hnu(N);
  rc = objective_weights(ctx, mu, ord, dord, dB, a, nullptr);
  const KParams K = ctx->kparams();
  if (rc == SESM_OK) {
    (void)hipMemcpyAsync(da, a.data(), sizeof(cplx) * no, hipMemcpyHostToDevice, ctx->stream);
    (void)hipMemcpyAsync(hnu.data(), nu, sizeof(cplx) * N, hipMemcpyDeviceToHost, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& v : hnu) v.im = -v.im;
    (void)hipMemcpyAsync(cnu, hnu.data(), sizeof(cplx) * N, hipMemcpyHostToDevice, ctx->stream);
    if (!kept)
      hipLaunchKernelGGL(k_dense_deriv, dim3((N + 3) / 4, N), dim3(256), 0, ctx->stream, K, ctx->x, ctx->f,
                         ctx->fp, ctx->fpp, ctx->J, ctx->logw, DY, DF);
    hipLaunchKernelGGL(k_gemv_rows_g, dim3(N), dim3(256), 0, ctx->stream, N, DY, mu, DYmu);
    hipLaunchKernelGGL(k_gemv_cols<false>, dim3((N + 63) / 64), dim3(1024), 0, ctx->stream, N, DY, cnu, DYtnu);
    hipLaunchKernelGGL(k_gemv_cols<false>, dim3((N + 63) / 64), dim3(1024), 0, ctx->stream, N, DF, cnu, DFtnu);
    hipLaunchKernelGGL(k_grad_nodes, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, K, no, dord, da, P.beta,
                       ctx->x, ctx->f, ctx->fp, ctx->fpp, ctx->J, mu, nu, DYmu, DYtnu, DFtnu, Pk, Qk, Rk);
    hipLaunchKernelGGL(k_grad_modes, dim3(2 * (n_modes + 1)), dim3(256), 0, ctx->stream, N, P.d, ctx->x, Pk, Qk, Rk,
                       dga, dgb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, std::string("shape gradient: ") + hipGetErrorString(e));
  }
  if (rc == SESM_OK) {
    (void)hipMemcpyAsync(grad_a, dga, sizeof(double) * (n_modes + 1), hipMemcpyDeviceToHost, ctx->stream);
    (void)hipMemcpyAsync(grad_b, dgb, sizeof(double) * (n_modes + 1), hipMemcpyDeviceToHost, ctx->stream);
  }
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (rc == SESM_OK && es != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(es));
  return rc;
}

// Dense set-up with sesm_params.adjoint = 1: the operator and its derivative
// matrices in one pass, all three kept with the surface.
int sesm_dense_assemble_with_derivs(sesm_ctx* ctx) {
  const Problem& P = ctx->P;
  const size_t NN = (size_t)P.N * P.N;
  int rc;
  if ((rc = sesm_alloc(ctx, (void**)&ctx->dA_dY, sizeof(cplx) * NN)) ||
      (rc = sesm_alloc(ctx, (void**)&ctx->dA_dF, sizeof(cplx) * NN)))
    return rc;
  const KParams K = ctx->kparams();
  hipLaunchKernelGGL(k_dense_assemble_deriv, dim3((P.N + 3) / 4, P.N), dim3(256), 0, ctx->stream, K, ctx->x, ctx->f,
                     ctx->fp, ctx->fpp, ctx->J, ctx->logw, ctx->Mdense, ctx->dA_dY, ctx->dA_dF);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

// y = (1/2 I + D^dx)^H mu (dense mode)
int sesm_dense_matvec_adjoint(sesm_ctx* ctx, const cplx* mu, cplx* y) {
  const int N = ctx->P.N;
  hipLaunchKernelGGL(k_gemv_cols<true>, dim3((N + 63) / 64), dim3(1024), 0, ctx->stream, N, ctx->Mdense, mu, y);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

extern "C" int sesm_matvec_adjoint(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_DENSE) return ctx->fail(SESM_EINVAL, "the adjoint map needs the dense mode");
  if (!mu || !y) return ctx->fail(SESM_EINVAL, "null pointer");
  if ((const void*)mu == (const void*)y) return ctx->fail(SESM_EINVAL, "mu and y must not overlap");
  SESM_HIP(hipSetDevice(ctx->device));
  return sesm_dense_matvec_adjoint(ctx, (const cplx*)mu, (cplx*)y);
}
