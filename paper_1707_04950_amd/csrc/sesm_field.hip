// Scattered field off the surface (sesm_field): the representation of eq.
// (eq:int_eq_dirichlet) evaluated at given points from a density mu.
//
// Three routes, chosen per point:
//  * accelerated mode, points inside the accelerator's cell grid: the
//    forward map's own stages (the remark closing Sec. 5.7), in
//    sesm_accel.hip;
//  * accelerated mode, points at least L/4 above the highest surface point:
//    the Rayleigh expansion u = sum_n B_n e^{i alpha_n x + i beta_n y} with
//    every order whose term can still matter (propagating and evanescent);
//  * every other point, and every point in dense mode: the trapezoidal rule of
//    the windowed lattice sums (eq. Gq_limit with the Bloch phase) over all
//    nodes, plus the completion modes (eq. M_eta) - the rule of eq. DAdx_def
//    without the singular split, which a point off the curve does not need.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sesm.h"
#include "sesm_impl.h"
#include "sesm_kernels.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

// Direct rule: one workgroup per point; threads over the nodes, the images p
// with S_{cA,A}(X_p) > 0 of each, the completion modes; fixed-order block sum.
__global__ __launch_bounds__(256) void k_field_direct(KParams K, const int* __restrict__ idx,
                                                      const double* __restrict__ px, const double* __restrict__ py,
                                                      const int* __restrict__ pp, const double* __restrict__ x,
                                                      const double* __restrict__ f, const double* __restrict__ fp,
                                                      const double* __restrict__ J, const cplx* __restrict__ mu,
                                                      cplx* __restrict__ u) {
  __shared__ cplx red[256];
  const int t = blockIdx.x;
  const double X = px[t], Y = py[t];
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < K.N; l += 256) {
    const double Xl = X - x[l], Yl = Y - f[l];
    const int p0 = (int)ceil((Xl - K.A_len) / K.d), p1 = (int)floor((Xl + K.A_len) / K.d);
    cplx s = cplx{0.0, 0.0};
    for (int p = p0; p <= p1; ++p) {
      const double Xp = Xl - p * K.d;
      const double S = sesm_window(Xp, K.cA, K.A_len);
      if (S == 0.0) continue;
      s += (S * cexp_i(K.alpha * K.d * p)) * sesm_kdl(K, Xp, Yl, fp[l]);
    }
    for (int n = 0; n < K.nU; ++n)
      s += (J[l] * exp(-K.Ubi[n] * Yl)) * cexp_i(K.Ua[n] * Xl + K.Ubr[n] * Yl);
    acc += (K.dx * mu[l]) * s;
  }
  const cplx sm = block_sum<256>(acc, red);
  if (threadIdx.x == 0) u[idx[t]] = cexp_i(K.alpha * K.d * pp[t]) * sm;
}

// (1 - e^{i beta h})^j / beta, j >= 1: as written for |beta| >= 1/2; for
// smaller |beta| through 1 - e^{i beta h} = -2i sin(beta h / 2) e^{i beta h / 2},
//   = (-2i)^j sin^{j-1}(beta h / 2) (h / 2) sinc(beta h / 2) e^{i j beta h / 2}.
__device__ inline cplx shift_quotient_dev(cplx beta, double h, int j) {
  auto cexpi = [](cplx z) {  // e^{i z}
    double sn, cs;
    sincos(z.re, &sn, &cs);
    const double m = exp(-z.im);
    return cplx{m * cs, m * sn};
  };
  if (abs2(beta) >= 0.25) {
    cplx one_m = cplx{1.0, 0.0} - cexpi(h * beta), pw = cplx{1.0, 0.0};
    for (int m = 0; m < j; ++m) pw = pw * one_m;
    return (1.0 / abs2(beta)) * cmul_conj(beta, pw);
  }
  const cplx z = (0.5 * h) * beta;
  double sn, cs;
  sincos(z.re, &sn, &cs);
  const cplx sz = cplx{sn * cosh(z.im), cs * sinh(z.im)};
  cplx sinc;
  if (abs2(z) < 1e-6) {
    const cplx z2 = z * z;
    sinc = cplx{1.0, 0.0} - (1.0 / 6.0) * z2 + (1.0 / 120.0) * (z2 * z2);
  } else {
    sinc = (1.0 / abs2(z)) * cmul_conj(z, sz);
  }
  cplx pw = (0.5 * h) * sinc;
  for (int m = 1; m < j; ++m) pw = pw * sz;
  cplx c2 = cplx{1.0, 0.0};
  for (int m = 0; m < j; ++m) c2 = cplx{2.0 * c2.im, -2.0 * c2.re};  // (-2i)^j
  return c2 * pw * cexpi((double)j * z);
}

// Rayleigh coefficients of all orders n = -nR..nR, referred to the height
// y_ref >= max f so that no evanescent factor overflows:
//   B~_n = dx sum_l [-(alpha_n f'_l - beta_n) Q_n / (2d) + 1[n in U] J_l] e^{-i alpha_n x_l - i beta_n (f_l - y_ref)} mu_l
// (Q_n = (1 - e^{i beta_n h})^j / beta_n).  One workgroup per order.
__global__ __launch_bounds__(256) void k_field_ray_coef(KParams K, int nR, double yref, const double* __restrict__ x,
                                                        const double* __restrict__ f, const double* __restrict__ fp,
                                                        const double* __restrict__ J, const cplx* __restrict__ mu,
                                                        cplx* __restrict__ B) {
  __shared__ cplx red[256];
  const int n = (int)blockIdx.x - nR;
  const double an = K.alpha + 2.0 * kPi * n / K.d;
  const double g = (K.k - an) * (K.k + an);
  const cplx bn = g >= 0.0 ? cplx{sqrt(g), 0.0} : cplx{0.0, sqrt(-g)};
  const cplx Q = shift_quotient_dev(bn, K.h, K.j);
  bool inU = false;
  for (int t = 0; t < K.nU; ++t) inU = inU || fabs(K.Ua[t] - an) <= 1e-9 * K.k;
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < K.N; l += 256) {
    cplx dl = (-1.0 / (2.0 * K.d)) * (cplx{an * fp[l] - bn.re, -bn.im} * Q);
    if (inU) dl.re += J[l];
    const double ph = -an * x[l] - bn.re * (f[l] - yref);
    const double mag = exp(bn.im * (f[l] - yref));
    acc += (mag * cexp_i(ph)) * (dl * mu[l]);
  }
  const cplx s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) B[blockIdx.x] = K.dx * s;
}

// u = e^{i alpha d p} sum_n B~_n e^{i alpha_n x + i beta_n (y - y_ref)}, one thread per point
__global__ void k_field_ray_eval(KParams K, int n_pts, int nR, double yref, const int* __restrict__ idx,
                                 const double* __restrict__ px, const double* __restrict__ py,
                                 const int* __restrict__ pp, const cplx* __restrict__ B, cplx* __restrict__ u) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pts) return;
  const double X = px[t], Yr = py[t] - yref;
  cplx acc = cplx{0.0, 0.0};
  for (int i = 0; i <= 2 * nR; ++i) {
    const double an = K.alpha + 2.0 * kPi * (i - nR) / K.d;
    const double g = (K.k - an) * (K.k + an);
    const double br = g >= 0.0 ? sqrt(g) : 0.0, bi = g >= 0.0 ? 0.0 : sqrt(-g);
    acc += (exp(-bi * Yr) * cexp_i(an * X + br * Yr)) * B[i];
  }
  u[idx[t]] = cexp_i(K.alpha * K.d * pp[t]) * acc;
}

}  // namespace

extern "C" int sesm_field(sesm_ctx* ctx, const sesm_c64* mu_, int32_t n, const double* xy, sesm_c64* u_) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (n < 0 || n > (1 << 24)) return ctx->fail(SESM_EINVAL, "field: number of points must be in [0, 2^24]");
  if (n == 0) return SESM_OK;
  if (!mu_ || !xy || !u_) return ctx->fail(SESM_EINVAL, "null pointer");
  SESM_HIP(hipSetDevice(ctx->device));
  const cplx* mu = reinterpret_cast<const cplx*>(mu_);
  cplx* u = reinterpret_cast<cplx*>(u_);
  const Problem& P = ctx->P;
  std::vector<double> hxy(2 * (size_t)n), hf(P.N);
  SESM_HIP(hipMemcpyAsync(hxy.data(), xy, sizeof(double) * 2 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipMemcpyAsync(hf.data(), ctx->f, sizeof(double) * P.N, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < hxy.size(); ++i)
    if (!std::isfinite(hxy[i])) return ctx->fail(SESM_EINVAL, "field: non-finite point coordinate");
  const double fmax = *std::max_element(hf.begin(), hf.end());
  const bool acc = P.mode == SESM_MODE_ACCEL;
  AccelGrid G{};
  double x0 = 0.0;
  if (acc) {
    G = sesm_accel_grid(ctx);
    x0 = G.x0;
  }
  const double dR = acc ? 0.25 * G.L : 0.0;
  // route and quasi-periodic shift of each point: x = x' + p d, x' in [x0, x0 + d)
  std::vector<int> ids[3], ps[3];
  std::vector<double> xs[3], ys[3];
  double dmin = 1e300;
  for (int t = 0; t < n; ++t) {
    const double X = hxy[2 * (size_t)t], Y = hxy[2 * (size_t)t + 1];
    const double pf = std::floor((X - x0) / P.d);
    if (std::fabs(pf) > 1e9) return ctx->fail(SESM_EINVAL, "field: point too far along the period");
    const int p = (int)pf;
    const double Xw = X - p * P.d;
    int r = 0;  // direct
    if (acc && Y >= G.y0 && Y < G.y0 + G.n_y * G.L) r = 1;
    else if (acc && Y >= fmax + dR) r = 2;
    if (r == 2) dmin = std::min(dmin, Y - fmax);
    ids[r].push_back(t);
    ps[r].push_back(p);
    xs[r].push_back(Xw);
    ys[r].push_back(Y);
  }
  int rc = SESM_OK;
  // points inside the cell grid: the accelerator's stages
  if (!ids[1].empty())
    rc = sesm_accel_field_cells(ctx, mu, (int)ids[1].size(), ids[1].data(), xs[1].data(), ys[1].data(),
                                ps[1].data(), u);
  if (rc) return rc;
  const KParams K = ctx->kparams();
  // Rayleigh orders: terms below e^{-40} of the largest once |beta_n| (y - max f) > 40
  int nR = 0;
  if (!ids[2].empty()) {
    const double need = std::sqrt((40.0 / dmin) * (40.0 / dmin) + P.k * P.k) + P.k;
    nR = (int)std::ceil(need * P.d / (2.0 * kPi)) + 2;
  }
  const size_t nd = ids[0].size(), nr = ids[2].size();
  const size_t bytes = (sizeof(int) * 2 + sizeof(double) * 2) * (nd + nr) + sizeof(cplx) * (2 * (size_t)nR + 1) + 256;
  char* buf = nullptr;
  SESM_HIP(hipMalloc((void**)&buf, bytes));
  char* cur = buf;
  auto put = [&](const void* src, size_t b) -> void* {
    void* d = cur;
    if (b) (void)hipMemcpyAsync(d, src, b, hipMemcpyHostToDevice, ctx->stream);
    cur += (b + 15) / 16 * 16;
    return d;
  };
  if (nd) {
    const int* di = (const int*)put(ids[0].data(), sizeof(int) * nd);
    const int* dp = (const int*)put(ps[0].data(), sizeof(int) * nd);
    const double* dx = (const double*)put(xs[0].data(), sizeof(double) * nd);
    const double* dy = (const double*)put(ys[0].data(), sizeof(double) * nd);
    hipLaunchKernelGGL(k_field_direct, dim3((unsigned)nd), dim3(256), 0, ctx->stream, K, di, dx, dy, dp, ctx->x,
                       ctx->f, ctx->fp, ctx->J, mu, u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, std::string("k_field_direct: ") + hipGetErrorString(e));
  }
  if (rc == SESM_OK && nr) {
    const int* di = (const int*)put(ids[2].data(), sizeof(int) * nr);
    const int* dp = (const int*)put(ps[2].data(), sizeof(int) * nr);
    const double* dx = (const double*)put(xs[2].data(), sizeof(double) * nr);
    const double* dy = (const double*)put(ys[2].data(), sizeof(double) * nr);
    cplx* B = (cplx*)cur;
    hipLaunchKernelGGL(k_field_ray_coef, dim3(2 * nR + 1), dim3(256), 0, ctx->stream, K, nR, fmax, ctx->x, ctx->f,
                       ctx->fp, ctx->J, mu, B);
    hipLaunchKernelGGL(k_field_ray_eval, dim3((unsigned)((nr + 127) / 128)), dim3(128), 0, ctx->stream, K, (int)nr,
                       nR, fmax, di, dx, dy, dp, B, u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, std::string("field (Rayleigh): ") + hipGetErrorString(e));
  }
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (rc == SESM_OK && es != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(es));
  return rc;
}
