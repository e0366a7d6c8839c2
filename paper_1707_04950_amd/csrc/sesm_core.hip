// Context, surface set-up (Algorithm 2), right-hand side, Rayleigh
// coefficients and efficiencies, and the operator dispatch.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "sesm_impl.h"

namespace {

constexpr double PI = 3.14159265358979323846;

// x_l = l d/N and f, f', f'' of the trigonometric profile at x_l.
__global__ void k_surface(int N, double d, int nm, const double* __restrict__ a, const double* __restrict__ b,
                          double* x, double* f, double* fp, double* fpp, double* J) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  const double xl = (double)l * (d / (double)N);
  double v = a[0], v1 = 0.0, v2 = 0.0;
  for (int m = 1; m <= nm; ++m) {
    const double w = 2.0 * PI * (double)m / d;
    double s, c;
    sincos(w * xl, &s, &c);
    v += a[m] * c + b[m] * s;
    v1 += w * (-a[m] * s + b[m] * c);
    v2 += -w * w * (a[m] * c + b[m] * s);
  }
  x[l] = xl;
  f[l] = v;
  fp[l] = v1;
  fpp[l] = v2;
  J[l] = sqrt(1.0 + v1 * v1);
}

// b_l = -exp(i (alpha x_l - beta f_l)), the Dirichlet data -u^inc of eq. (fist_eq).
__global__ void k_rhs(int N, double alpha, double beta, const double* __restrict__ x, const double* __restrict__ f,
                      cplx* b) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= N) return;
  const cplx e = cexp_i(alpha * x[l] - beta * f[l]);
  b[l] = cplx{-e.re, -e.im};
}

struct OrderCoef {
  double an, br, bi;  // alpha_n, beta_n = br + i bi
  double qr, qi;      // (1 - e^{i beta_n h})^j / beta_n
  int inU;            // n in U^eta
  int pad;
};

// B_n = dx sum_l [ -(alpha_n f'_l - beta_n) Q_n / (2d) + 1[n in U^eta] J_l ]
//                * exp(-i alpha_n x_l - i beta_n f_l) mu_l      (one block per order)
__global__ void k_rayleigh(int N, double d, double dx, const OrderCoef* __restrict__ oc,
                           const double* __restrict__ x, const double* __restrict__ f,
                           const double* __restrict__ fp, const double* __restrict__ J,
                           const cplx* __restrict__ mu, cplx* B) {
  __shared__ cplx sh[4];
  const OrderCoef o = oc[blockIdx.x];
  const cplx Q = cplx{o.qr, o.qi};
  const cplx bn = cplx{o.br, o.bi};
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < N; l += blockDim.x) {
    // -(alpha_n f' - beta_n) Q / (2d)
    const cplx g = cplx{-o.an * fp[l] + bn.re, bn.im};
    cplx kern = (1.0 / (2.0 * d)) * (g * Q);
    if (o.inU) kern.re += J[l];
    // exp(-i alpha_n x - i beta_n f) = exp(bi f) exp(-i (alpha_n x + br f))
    const double mag = exp(o.bi * f[l]);
    const cplx e = cexp_i(-(o.an * x[l] + o.br * f[l]));
    acc += (mag * (kern * e)) * mu[l];
  }
  const cplx s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) B[blockIdx.x] = dx * s;
}

__global__ void k_diag_hankel(int n, const double* __restrict__ x, cplx* h0, cplx* h1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cplx a, b;
  sesm_hankel01(x[i], &a, &b);
  h0[i] = a;
  h1[i] = b;
}

__global__ void k_diag_cexp(int n, const double* __restrict__ t, cplx* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = cexp_i_reduced(t[i]);
}

double binom(int n, int m) {
  double r = 1.0;
  for (int t = 1; t <= m; ++t) r = r * (double)(n - m + t) / (double)t;
  return r;
}

std::complex<double> beta_of(double k, double an) {
  const double disc = k * k - an * an;
  return disc >= 0 ? std::complex<double>(std::sqrt(std::fabs(disc)), 0.0)
                   : std::complex<double>(0.0, std::sqrt(std::fabs(disc)));
}

// (1 - e^{i beta h})^j / beta with 1 - e^{iz} = -2i sin(z/2) e^{iz/2}
std::complex<double> shift_quotient(std::complex<double> b, double h, int j) {
  if (b == 0.0) {
    if (j >= 2) return 0.0;
    if (j == 1) return std::complex<double>(0.0, -h);
    return std::complex<double>(INFINITY, 0.0);
  }
  const std::complex<double> z = b * h;
  const std::complex<double> I(0.0, 1.0);
  return std::pow(-2.0 * I, j) * std::pow(std::sin(z / 2.0), j) * std::exp(0.5 * (double)j * I * z) / b;
}

}  // namespace

// The incidence-dependent scalars of a problem whose d, k, j and h are set:
// alpha, beta, the completion set U^eta with its alpha_n, beta_n, and the
// propagating orders.  False if U^eta has more than SESM_MAX_UETA members.
bool sesm_problem_alpha(Problem& P, double alpha, double eta) {
  const double d = P.d, k = P.k, h = P.h;
  const int j = P.j;
  P.alpha = alpha;
  P.beta = std::sqrt(std::max(0.0, k * k - alpha * alpha));
  // U^eta = {n : |1 - e^{i beta_n h}|^j < eta} (eq. M_eta).  The printed set, with the
  // factor 1/beta_n, is infinite (the quotient tends to zero for evanescent
  // orders); on a flat surface 1/2 I + D~ has the eigenvalue (1/2)(1 - e^{i beta_n h})^j
  // on e^{i alpha_n x}, so the orders where that factor is small are the ones
  // the completion modes must restore.
  P.nU = 0;
  if (j > 0) {
    const double t = std::pow(eta, 1.0 / j);
    const double kmax = -std::log(1.0 - std::min(t, 0.999999)) / h + 1.0;
    const double K = std::sqrt(k * k + kmax * kmax);
    const int nlo = (int)std::floor((-K - alpha) * d / (2 * PI)) - 1;
    const int nhi = (int)std::ceil((K - alpha) * d / (2 * PI)) + 1;
    for (int n = nlo; n <= nhi; ++n) {
      const double an = alpha + 2.0 * PI * n / d;
      const std::complex<double> b = beta_of(k, an);
      const double fac = std::pow(std::abs(1.0 - std::exp(std::complex<double>(0.0, 1.0) * b * h)), j);
      if (fac < eta) {
        if (P.nU >= SESM_MAX_UETA) return false;
        P.U[P.nU] = n;
        P.Ua[P.nU] = an;
        P.Ubr[P.nU] = b.real();
        P.Ubi[P.nU] = b.imag();
        ++P.nU;
      }
    }
  }
  const int nlo = (int)std::floor((-k - alpha) * d / (2 * PI)) - 1;
  const int nhi = (int)std::ceil((k - alpha) * d / (2 * PI)) + 1;
  int first = 0, count = 0;
  for (int n = nlo; n <= nhi; ++n) {
    const double an = alpha + 2.0 * PI * n / d;
    if (k * k - an * an > 0) {
      if (count == 0) first = n;
      ++count;
    }
  }
  P.n_first = first;
  P.n_count = count;
  return true;
}

// keeps released blocks for the next surface up to this many bytes
static constexpr size_t kPoolLimit = (size_t)16 << 30;

static void pool_drain(sesm_ctx* ctx) {
  for (auto& b : ctx->pool) (void)hipFree(b.second);
  ctx->pool.clear();
  ctx->pool_bytes = 0;
}

void sesm_pool_put(sesm_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  if (ctx->pool_bytes + bytes > kPoolLimit) {
    (void)hipFree(p);
    return;
  }
  ctx->pool.emplace_back(bytes, p);
  ctx->pool_bytes += bytes;
}

int sesm_alloc(sesm_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  for (size_t t = 0; t < ctx->pool.size(); ++t)  // a released block of exactly this size
    if (ctx->pool[t].first == bytes) {
      *p = ctx->pool[t].second;
      ctx->pool[t] = ctx->pool.back();
      ctx->pool.pop_back();
      ctx->pool_bytes -= bytes;
      break;
    }
  if (!*p) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess && !ctx->pool.empty()) {  // give the pool back and try again
      (void)hipGetLastError();
      pool_drain(ctx);
      e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return ctx->fail(SESM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
  }
  ctx->owned.emplace_back(*p, bytes);
  ctx->bytes += (int64_t)bytes;
  if (ctx->poison &&  // every byte 0xFF: a NaN in each double, so a read before the first write shows
      (hipMemsetAsync(*p, 0xFF, bytes, ctx->stream) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess))
    return ctx->fail(SESM_EHIP, "poisoning an allocation failed");
  return SESM_OK;
}

void sesm_release_surface(sesm_ctx* ctx) {
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  sesm_accel_free(ctx);
  for (auto& o : ctx->owned) sesm_pool_put(ctx, o.first, o.second);
  ctx->owned.clear();
  ctx->bytes = 0;
  ctx->x = ctx->f = ctx->fp = ctx->fpp = ctx->J = ctx->logw = nullptr;
  ctx->Mdense = ctx->dA_dY = ctx->dA_dF = nullptr;
  ctx->V = nullptr;
  ctx->V_cols = 0;
  ctx->hcol = ctx->hpart = ctx->ybuf = ctx->wtmp = ctx->gw = ctx->Hrow = ctx->htri = ctx->hp = ctx->gcoef = nullptr;
  ctx->gsc = nullptr;
  ctx->umix = ctx->mx_r = ctx->mx_R = ctx->mx_D = nullptr;
  ctx->ray_oc = nullptr;
  ctx->ray_B = nullptr;
  ctx->ray_cap = 0;
  ctx->Hrow_len = 0;
  ctx->Hrow_m = -1;
  ctx->ready = false;  // (the pinned column slots stay: they do not depend on the surface)
}

KParams sesm_ctx::kparams() const {
  KParams K{};
  K.N = P.N;
  K.j = P.j;
  K.n_a = P.n_a;
  K.pmin = P.pmin;
  K.pmax = P.pmax;
  K.nU = P.nU;
  K.d = P.d;
  K.k = P.k;
  K.alpha = P.alpha;
  K.dx = P.dx;
  K.h = P.h;
  K.A_len = P.A_len;
  K.cA = P.cA;
  K.a = P.a;
  K.gamma = P.gamma;
  for (int m = 0; m <= SESM_MAX_J; ++m) K.wshift[m] = P.wshift[m];
  for (int t = 0; t < SESM_MAX_UETA; ++t) {
    K.Ua[t] = P.Ua[t];
    K.Ubr[t] = P.Ubr[t];
    K.Ubi[t] = P.Ubi[t];
  }
  return K;
}

// Per-order constants of k_rayleigh: alpha_n, beta_n, (1 - e^{i beta_n h})^j / beta_n
// and membership in U^eta.
static int order_constants(sesm_ctx* ctx, const int32_t* orders, int n_orders, OrderCoef* oc) {
  const Problem& P = ctx->P;
  for (int t = 0; t < n_orders; ++t) {
    const int n = orders[t];
    const double an = P.alpha + 2.0 * PI * n / P.d;
    const std::complex<double> b = beta_of(P.k, an);
    const std::complex<double> q = shift_quotient(b, P.h, P.j);
    oc[t].an = an;
    oc[t].br = b.real();
    oc[t].bi = b.imag();
    oc[t].qr = q.real();
    oc[t].qi = q.imag();
    oc[t].inU = 0;
    oc[t].pad = 0;
    for (int u = 0; u < P.nU; ++u)
      if (P.U[u] == n) oc[t].inU = 1;
    if (!std::isfinite(q.real()) || !std::isfinite(q.imag()))
      return ctx->fail(SESM_EINVAL, "Rayleigh coefficient undefined (Wood order with j = 0)");
  }
  return SESM_OK;
}

// ---------------------------------------------------------------------------
// Fixed device array for sesm_rayleigh_noalloc: the constants of up to
// SESM_RAYLEIGH_NOALLOC_MAX orders, then their results.  Host code never uses
// the array's name as an address: each device's copy is looked up once
// (hipGetSymbolAddress, at the first sesm_create on that device) and only
// that pointer is handed to kernels and copies.
#define SESM_NOALLOC_DEVICES 64
static __device__ __align__(256) unsigned char scratch[(size_t)SESM_RAYLEIGH_NOALLOC_MAX * (sizeof(OrderCoef) + sizeof(cplx))];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SESM_NOALLOC_DEVICES] = {};

// the device address of `scratch` on the current device `device`
static hipError_t scratch_lookup(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= SESM_NOALLOC_DEVICES) {
    *out = nullptr;
    return hipSuccess;  // (the entry point then reports that it is unavailable)
  }
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// device room for the constants and results of n Rayleigh orders
static int rayleigh_buffers(sesm_ctx* ctx, int n) {
  int rc;
  void* oc = nullptr;
  cplx* B = nullptr;
  if ((rc = sesm_alloc(ctx, &oc, sizeof(OrderCoef) * (size_t)n)) || (rc = sesm_alloc(ctx, (void**)&B, sizeof(cplx) * (size_t)n)))
    return rc;
  ctx->ray_oc = oc;  // (an earlier, smaller pair stays owned by the surface)
  ctx->ray_B = B;
  ctx->ray_cap = n;
  return SESM_OK;
}

int sesm_apply(sesm_ctx* ctx, const cplx* mu, cplx* y) {
  if (ctx->P.mode == SESM_MODE_ACCEL) return sesm_accel_matvec(ctx, mu, y);
  return sesm_dense_matvec(ctx, mu, y);
}

int sesm_apply_inc(sesm_ctx* ctx, const cplx* mu, cplx* y, int inc, bool mixed) {
  if (mixed && ctx->P.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "mixed precision needs the accelerated mode");
  if (inc < 0) return ctx->P.mode == SESM_MODE_ACCEL ? sesm_accel_matvec(ctx, mu, y, mixed) : sesm_dense_matvec(ctx, mu, y);
  return sesm_accel_matvec_batch(ctx, 1, mu, ctx->P.N, y, ctx->P.N, inc, mixed);
}

// checks shared by the incidence-set entry points
static int incidence_ready(sesm_ctx* ctx, int r0, int n) {
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "incidence sets need the accelerated mode");
  const int ni = sesm_accel_n_incidences(ctx);
  if (r0 < 0 || n < 0 || r0 + n > ni) return ctx->fail(SESM_EINVAL, "incidence index beyond the incidence set");
  return SESM_OK;
}

extern "C" {

int sesm_create(sesm_ctx** out, int device, void* hip_stream) {
  if (!out) return SESM_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SESM_EHIP;
  }
  if (hipSetDevice(device) != hipSuccess) return SESM_EHIP;
  sesm_ctx* ctx = new (std::nothrow) sesm_ctx();
  if (!ctx) return SESM_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (scratch_lookup(device, &ctx->noalloc_scratch) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return SESM_EHIP;
  }
  const char* pv = std::getenv("SESM_POISON_ALLOC");
  ctx->poison = pv && pv[0] && pv[0] != '0';
  *out = ctx;
  return SESM_OK;
}

int sesm_destroy(sesm_ctx* ctx) {
  if (!ctx) return SESM_OK;
  (void)hipSetDevice(ctx->device);
  sesm_release_surface(ctx);
  pool_drain(ctx);
  if (ctx->hhost) (void)hipHostFree(ctx->hhost);
  if (ctx->hflag) (void)hipHostFree(ctx->hflag);
  sesm_kt_free(ctx);
  delete ctx;
  return SESM_OK;
}

const char* sesm_last_error(const sesm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sesm_set_surface(sesm_ctx* ctx, const sesm_profile* prof, double d, double k, double alpha, int32_t j,
                     double A_periods, const sesm_params* params) {
  if (!ctx) return SESM_EINVAL;
  ctx->err.clear();
  if (!prof || !params) return ctx->fail(SESM_EINVAL, "profile and params are required");
  if (prof->n_modes < 0 || prof->n_modes > 1 << 20 || !prof->a || (prof->n_modes > 0 && !prof->b))
    return ctx->fail(SESM_EINVAL, "invalid profile");
  for (int m = 0; m <= prof->n_modes; ++m)
    if (!std::isfinite(prof->a[m]) || (m > 0 && !std::isfinite(prof->b[m])))
      return ctx->fail(SESM_EINVAL, "non-finite profile coefficient");
  if (!(d > 0) || !std::isfinite(d) || !(k > 0) || !std::isfinite(k) || !std::isfinite(alpha))
    return ctx->fail(SESM_EINVAL, "d and k must be positive and finite");
  if (!(std::fabs(alpha) < k)) return ctx->fail(SESM_EINVAL, "need |alpha| < k (non-grazing incidence)");
  if (j < 0 || j > SESM_MAX_J) return ctx->fail(SESM_EINVAL, "shift order j must be in [0, 16]");
  if (!(A_periods > 0) || !std::isfinite(A_periods) || A_periods > 1e5)
    return ctx->fail(SESM_EINVAL, "window half-width A (periods) must be positive");
  sesm_params prm = *params;
  if (prm.N < 8 || prm.N > (1 << 26)) return ctx->fail(SESM_EINVAL, "N must be in [8, 2^26]");
  const double lambda = 2.0 * PI / k;
  if (prm.h == 0) prm.h = 0.5 * lambda;
  if (prm.c_window == 0) prm.c_window = 0.5;
  if (prm.gamma_frac == 0) prm.gamma_frac = 0.5;
  if (prm.eta == 0) prm.eta = 1e-3;
  if (prm.L_cell == 0) prm.L_cell = 0.5 * lambda;
  const double dx = d / prm.N;
  if (prm.n_a == 0) prm.n_a = std::max(8, (int)std::floor(0.8 * std::min(prm.L_cell, d) / dx));
  if (!(prm.h > 0) || !(prm.c_window > 0 && prm.c_window < 1) || !(prm.gamma_frac > 0 && prm.gamma_frac < 1) ||
      !(prm.eta > 0) || !(prm.L_cell > 0) || prm.n_a < 2)
    return ctx->fail(SESM_EINVAL, "invalid discretisation parameter");
  if (prm.mode != SESM_MODE_DENSE && prm.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "unknown mode");
  if (prm.table != 0 && prm.table != 1) return ctx->fail(SESM_EINVAL, "table must be 0 (windowed) or 1 (hybrid)");
  if (prm.adjoint != 0 && prm.adjoint != 1) return ctx->fail(SESM_EINVAL, "adjoint must be 0 or 1");
  if (prm.adjoint == 1 && prm.mode != SESM_MODE_DENSE)
    return ctx->fail(SESM_EINVAL, "adjoint = 1 (derivative matrices) needs the dense mode");
  if (prm.table == 1 && (prm.mode != SESM_MODE_ACCEL || j < 1))
    return ctx->fail(SESM_EINVAL, "hybrid tables need the accelerated mode and j >= 1");
  const double a = prm.n_a * dx;
  if (!(a < d)) return ctx->fail(SESM_EINVAL, "singular window a = n_a dx must be < d (Remark selec_a)");
  if (!(prm.c_window * A_periods * d > a)) return ctx->fail(SESM_EINVAL, "window plateau c A must exceed a");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(SESM_EHIP, "hipSetDevice failed");

  sesm_release_surface(ctx);
  ctx->prm = prm;
  Problem& P = ctx->P;
  P = Problem();
  P.N = prm.N;
  P.j = j;
  P.n_a = prm.n_a;
  P.mode = prm.mode;
  P.d = d;
  P.k = k;
  P.alpha = alpha;
  P.beta = std::sqrt(k * k - alpha * alpha);
  P.h = prm.h;
  P.A_len = A_periods * d;
  P.cA = prm.c_window * P.A_len;
  P.dx = dx;
  P.a = a;
  P.gamma = prm.gamma_frac * a;
  P.eta = prm.eta;
  for (int m = 0; m <= SESM_MAX_J; ++m) P.wshift[m] = (m <= j) ? ((m & 1) ? -1.0 : 1.0) * binom(j, m) : 0.0;
  P.pmax = (int)std::ceil(A_periods) + 1;
  P.pmin = -P.pmax;
  if (!sesm_problem_alpha(P, alpha, prm.eta)) return ctx->fail(SESM_EINVAL, "more than 64 completion modes; lower eta");

  // surface samples
  int rc;
  const size_t Nb = sizeof(double) * (size_t)P.N;
  if ((rc = sesm_alloc(ctx, (void**)&ctx->x, Nb)) || (rc = sesm_alloc(ctx, (void**)&ctx->f, Nb)) ||
      (rc = sesm_alloc(ctx, (void**)&ctx->fp, Nb)) || (rc = sesm_alloc(ctx, (void**)&ctx->fpp, Nb)) ||
      (rc = sesm_alloc(ctx, (void**)&ctx->J, Nb)))
    return rc;
  const int nm = prof->n_modes;
  std::vector<double> ab(2 * (size_t)(nm + 1), 0.0);
  for (int m = 0; m <= nm; ++m) {
    ab[m] = prof->a[m];
    ab[nm + 1 + m] = m > 0 ? prof->b[m] : 0.0;
  }
  double* dab = nullptr;
  if ((rc = sesm_alloc(ctx, (void**)&dab, sizeof(double) * ab.size()))) return rc;
  SESM_HIP(hipMemcpyAsync(dab, ab.data(), sizeof(double) * ab.size(), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_surface, dim3((P.N + 255) / 256), dim3(256), 0, ctx->stream, P.N, d, nm, dab, dab + nm + 1,
                     ctx->x, ctx->f, ctx->fp, ctx->fpp, ctx->J);
  SESM_LAUNCH_CHECK();
  // log-quadrature weights R_m, m = 0..n_a-1 (eq. local_mat):
  //   R_m = -2 dx sum_{s=1}^{n_a/2} w_s cos(2 pi s m / n_a) / s,  w_s = 1/2 if 2 s = n_a, else 1,
  // the trapezoidal weights that integrate ln(4 sin^2(pi t / a)) times a
  // trigonometric polynomial of degree n_a on the window period a exactly,
  // from int_{-a}^{a} ln(4 sin^2(pi t / a)) e^{i pi q t / a} dt = -4 a / |q| for
  // even q != 0 and 0 for odd q.
  {
    std::vector<double> R(P.n_a);
    for (int m = 0; m < P.n_a; ++m) {
      double s = 0.0;
      for (int q = 1; q <= P.n_a / 2; ++q) {
        const double w = (2 * q == P.n_a) ? 0.5 : 1.0;
        s += w * std::cos(2.0 * PI * q * m / P.n_a) / q;
      }
      R[m] = -2.0 * dx * s;
    }
    if ((rc = sesm_alloc(ctx, (void**)&ctx->logw, sizeof(double) * P.n_a))) return rc;
    SESM_HIP(hipMemcpyAsync(ctx->logw, R.data(), sizeof(double) * P.n_a, hipMemcpyHostToDevice, ctx->stream));
  }
  if ((rc = rayleigh_buffers(ctx, std::max(64, P.n_count)))) return rc;
  if (P.mode == SESM_MODE_DENSE) {
    if ((rc = sesm_dense_setup(ctx))) return rc;
  } else {
    if ((rc = sesm_accel_setup(ctx))) return rc;
  }
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  ctx->ready = true;
  return SESM_OK;
}

int sesm_get_info(const sesm_ctx* ctx, sesm_surface_info* info) {
  if (!ctx || !info) return SESM_EINVAL;
  if (!ctx->ready) return SESM_ENOSURF;
  std::memset(info, 0, sizeof(*info));
  const Problem& P = ctx->P;
  info->N = P.N;
  info->n_a = P.n_a;
  info->dx = P.dx;
  info->a = P.a;
  info->gamma = P.gamma;
  info->h = P.h;
  info->A_len = P.A_len;
  info->mode = P.mode;
  info->n_eta = P.nU;
  for (int t = 0; t < P.nU && t < 16; ++t) info->U_eta[t] = P.U[t];
  info->n_first = P.n_first;
  info->n_count = P.n_count;
  info->device_bytes = ctx->bytes + (int64_t)ctx->pool_bytes;
  if (P.mode == SESM_MODE_ACCEL) sesm_accel_info(ctx, info);
  return SESM_OK;
}

int sesm_matvec(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu || !y || (const void*)mu == (const void*)y) return ctx->fail(SESM_EINVAL, "invalid vectors");
  SESM_HIP(hipSetDevice(ctx->device));
  return sesm_apply(ctx, (const cplx*)mu, (cplx*)y);
}

int sesm_matvec_batch(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* mu, int64_t ld_mu, sesm_c64* y, int64_t ld_y) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (nrhs < 0) return ctx->fail(SESM_EINVAL, "negative number of densities");
  if (nrhs == 0) return SESM_OK;
  const int64_t N = ctx->P.N;
  if (!mu || !y) return ctx->fail(SESM_EINVAL, "null pointer");
  if (ld_mu < N || ld_y < N) return ctx->fail(SESM_EINVAL, "leading dimension below N");
  // the two spans [p, p + (nrhs - 1) ld + N) must be disjoint
  const uintptr_t m0 = (uintptr_t)mu, m1 = (uintptr_t)(mu + (nrhs - 1) * ld_mu + N);
  const uintptr_t y0 = (uintptr_t)y, y1 = (uintptr_t)(y + (nrhs - 1) * ld_y + N);
  if (m0 < y1 && y0 < m1) return ctx->fail(SESM_EINVAL, "densities and outputs overlap");
  SESM_HIP(hipSetDevice(ctx->device));
  if (ctx->P.mode == SESM_MODE_ACCEL) return sesm_accel_matvec_batch(ctx, nrhs, (const cplx*)mu, ld_mu, (cplx*)y, ld_y);
  for (int r = 0; r < nrhs; ++r) {
    const int rc = sesm_dense_matvec(ctx, (const cplx*)(mu + r * ld_mu), (cplx*)(y + r * ld_y));
    if (rc) return rc;
  }
  return SESM_OK;
}

int sesm_rhs_bloch(sesm_ctx* ctx, int32_t p, sesm_c64* b) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!b) return ctx->fail(SESM_EINVAL, "null vector");
  const Problem& P = ctx->P;
  const double PI_ = 3.14159265358979323846;
  const double ap = P.alpha + 2.0 * PI_ * p / P.d;
  if (!(std::fabs(ap) < P.k)) return ctx->fail(SESM_EINVAL, "Bloch-class incidence is not propagating (|alpha_p| >= k)");
  const double bp = std::sqrt(P.k * P.k - ap * ap);
  SESM_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_rhs, dim3((P.N + 255) / 256), dim3(256), 0, ctx->stream, P.N, ap, bp, ctx->x, ctx->f,
                     (cplx*)b);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

int sesm_rhs(sesm_ctx* ctx, sesm_c64* b) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!b) return ctx->fail(SESM_EINVAL, "null vector");
  SESM_HIP(hipSetDevice(ctx->device));
  const Problem& P = ctx->P;
  hipLaunchKernelGGL(k_rhs, dim3((P.N + 255) / 256), dim3(256), 0, ctx->stream, P.N, P.alpha, P.beta, ctx->x,
                     ctx->f, (cplx*)b);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

int sesm_rayleigh(sesm_ctx* ctx, const sesm_c64* mu, const int32_t* orders, int32_t n_orders, sesm_c64* B_host) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu || !orders || !B_host || n_orders < 0 || n_orders > 1 << 20) return ctx->fail(SESM_EINVAL, "bad args");
  if (n_orders == 0) return SESM_OK;
  SESM_HIP(hipSetDevice(ctx->device));
  const Problem& P = ctx->P;
  std::vector<OrderCoef> oc(n_orders);
  int rc = order_constants(ctx, orders, n_orders, oc.data());
  if (rc) return rc;
  // the surface's buffers hold the propagating orders; more orders than that
  // grow them once (owned by the surface like every other table)
  if (n_orders > ctx->ray_cap && (rc = rayleigh_buffers(ctx, n_orders))) return rc;
  OrderCoef* doc = (OrderCoef*)ctx->ray_oc;
  cplx* dB = ctx->ray_B;
  // the previous call's host copy has completed (each call synchronises), so
  // the constants can be overwritten in stream order
  SESM_HIP(hipMemcpyAsync(doc, oc.data(), sizeof(OrderCoef) * n_orders, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_rayleigh, dim3(n_orders), dim3(256), 0, ctx->stream, P.N, P.d, P.dx, doc, ctx->x, ctx->f,
                     ctx->fp, ctx->J, (const cplx*)mu, dB);
  SESM_LAUNCH_CHECK();
  hipError_t e1 = hipMemcpyAsync(B_host, dB, sizeof(cplx) * n_orders, hipMemcpyDeviceToHost, ctx->stream);
  hipError_t e2 = hipStreamSynchronize(ctx->stream);
  if (e1 != hipSuccess || e2 != hipSuccess)
    return ctx->fail(SESM_EHIP, std::string("rayleigh: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return SESM_OK;
}

int sesm_rayleigh_noalloc(sesm_ctx* ctx, const sesm_c64* mu, const int32_t* orders, int32_t n_orders,
                          sesm_c64* B_host) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu || !orders || !B_host || n_orders < 0) return ctx->fail(SESM_EINVAL, "bad args");
  if (n_orders > SESM_RAYLEIGH_NOALLOC_MAX)
    return ctx->fail(SESM_EINVAL, "sesm_rayleigh_noalloc: at most SESM_RAYLEIGH_NOALLOC_MAX (" +
                                      std::to_string(SESM_RAYLEIGH_NOALLOC_MAX) + ") orders per call");
  if (!ctx->noalloc_scratch) return ctx->fail(SESM_EINVAL, "sesm_rayleigh_noalloc: device index out of range");
  if (n_orders == 0) return SESM_OK;
  SESM_HIP(hipSetDevice(ctx->device));
  const Problem& P = ctx->P;
  std::vector<OrderCoef> oc(n_orders);
  int rc = order_constants(ctx, orders, n_orders, oc.data());
  if (rc) return rc;
  OrderCoef* doc = (OrderCoef*)ctx->noalloc_scratch;
  cplx* dB = (cplx*)((unsigned char*)ctx->noalloc_scratch + (size_t)SESM_RAYLEIGH_NOALLOC_MAX * sizeof(OrderCoef));
  SESM_HIP(hipMemcpyAsync(doc, oc.data(), sizeof(OrderCoef) * n_orders, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_rayleigh, dim3(n_orders), dim3(256), 0, ctx->stream, P.N, P.d, P.dx, doc, ctx->x, ctx->f,
                     ctx->fp, ctx->J, (const cplx*)mu, dB);
  SESM_LAUNCH_CHECK();
  hipError_t e1 = hipMemcpyAsync(B_host, dB, sizeof(cplx) * n_orders, hipMemcpyDeviceToHost, ctx->stream);
  hipError_t e2 = hipStreamSynchronize(ctx->stream);
  if (e1 != hipSuccess || e2 != hipSuccess)
    return ctx->fail(SESM_EHIP, std::string("rayleigh_noalloc: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return SESM_OK;
}

int sesm_efficiencies(sesm_ctx* ctx, const sesm_c64* mu, int32_t* n_first, int32_t* n_count, double* e_host,
                      int32_t e_capacity, double* energy_error) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu || !n_first || !n_count || (e_capacity > 0 && !e_host) || e_capacity < 0)
    return ctx->fail(SESM_EINVAL, "bad args");
  const Problem& P = ctx->P;
  std::vector<int32_t> ord(P.n_count);
  for (int t = 0; t < P.n_count; ++t) ord[t] = P.n_first + t;
  std::vector<sesm_c64> B(P.n_count);
  int rc = sesm_rayleigh(ctx, mu, ord.data(), P.n_count, B.data());
  if (rc) return rc;
  double s = 0.0;
  for (int t = 0; t < P.n_count; ++t) {
    const double an = P.alpha + 2.0 * PI * ord[t] / P.d;
    const double bn = std::sqrt(std::fabs(P.k * P.k - an * an));
    const double e = bn / P.beta * (B[t].re * B[t].re + B[t].im * B[t].im);
    s += e;
    if (t < e_capacity) e_host[t] = e;
  }
  *n_first = P.n_first;
  *n_count = P.n_count;
  if (energy_error) *energy_error = 1.0 - s;
  return SESM_OK;
}

int sesm_set_incidences(sesm_ctx* ctx, int32_t n, const double* alpha) {
  if (!ctx) return SESM_EINVAL;
  if (n < 0 || n > SESM_MAX_INCIDENCES || (n > 0 && !alpha)) return ctx->fail(SESM_EINVAL, "bad incidence set");
  int rc = incidence_ready(ctx, 0, 0);
  if (rc) return rc;
  SESM_HIP(hipSetDevice(ctx->device));
  return sesm_accel_set_incidences(ctx, n, alpha);
}

int sesm_rhs_incidence(sesm_ctx* ctx, int32_t r, sesm_c64* b) {
  if (!ctx) return SESM_EINVAL;
  int rc = incidence_ready(ctx, r, 1);
  if (rc) return rc;
  if (!b) return ctx->fail(SESM_EINVAL, "null vector");
  SESM_HIP(hipSetDevice(ctx->device));
  const Problem* Q = sesm_accel_incidence(ctx, r);
  hipLaunchKernelGGL(k_rhs, dim3((ctx->P.N + 255) / 256), dim3(256), 0, ctx->stream, ctx->P.N, Q->alpha, Q->beta,
                     ctx->x, ctx->f, (cplx*)b);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

int sesm_matvec_incidences(sesm_ctx* ctx, int32_t r0, int32_t nrhs, const sesm_c64* mu, int64_t ld_mu, sesm_c64* y,
                           int64_t ld_y) {
  if (!ctx) return SESM_EINVAL;
  int rc = incidence_ready(ctx, r0, nrhs);
  if (rc) return rc;
  if (nrhs == 0) return SESM_OK;
  const int64_t N = ctx->P.N;
  if (!mu || !y) return ctx->fail(SESM_EINVAL, "null pointer");
  if (ld_mu < N || ld_y < N) return ctx->fail(SESM_EINVAL, "leading dimension below N");
  const uintptr_t m0 = (uintptr_t)mu, m1 = (uintptr_t)(mu + (nrhs - 1) * ld_mu + N);
  const uintptr_t y0 = (uintptr_t)y, y1 = (uintptr_t)(y + (nrhs - 1) * ld_y + N);
  if (m0 < y1 && y0 < m1) return ctx->fail(SESM_EINVAL, "densities and outputs overlap");
  SESM_HIP(hipSetDevice(ctx->device));
  return sesm_accel_matvec_batch(ctx, nrhs, (const cplx*)mu, ld_mu, (cplx*)y, ld_y, r0);
}

int sesm_efficiencies_incidence(sesm_ctx* ctx, int32_t r, const sesm_c64* mu, int32_t* n_first, int32_t* n_count,
                                double* e_host, int32_t e_capacity, double* energy_error) {
  if (!ctx) return SESM_EINVAL;
  int rc = incidence_ready(ctx, r, 1);
  if (rc) return rc;
  // the Rayleigh coefficients of member r: the problem's scalars with its alpha
  const Problem saved = ctx->P;
  ctx->P = *sesm_accel_incidence(ctx, r);
  rc = sesm_efficiencies(ctx, mu, n_first, n_count, e_host, e_capacity, energy_error);
  ctx->P = saved;
  return rc;
}

int sesm_diag_hankel(sesm_ctx* ctx, const double* x, int32_t n, sesm_c64* h0, sesm_c64* h1) {
  if (!ctx) return SESM_EINVAL;
  if (!x || !h0 || !h1 || n < 0) return ctx->fail(SESM_EINVAL, "bad args");
  if (n == 0) return SESM_OK;
  SESM_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_diag_hankel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, x, (cplx*)h0, (cplx*)h1);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

int sesm_diag_cexp(sesm_ctx* ctx, const double* t, int32_t n, sesm_c64* out) {
  if (!ctx) return SESM_EINVAL;
  if (!t || !out || n < 0) return ctx->fail(SESM_EINVAL, "bad args");
  if (n == 0) return SESM_OK;
  SESM_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_diag_cexp, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, t, (cplx*)out);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// per-kernel timing

static const char* const kKtNames[SESM_KT_COUNT] = {
    "k_local_apply", "k_merge_fft", "k_fft_rows",    "k_yconv",    "k_cells_far",
    "k_gm_dots",     "k_gm_update",   "k_gemv_rows"};

static int kt_fold(sesm_ctx* ctx, KTimer& T) {
  if (T.used == 0) return SESM_OK;
  SESM_HIP(hipEventSynchronize(T.ev[2 * T.used - 1]));
  for (int u = 0; u < T.used; ++u) {
    SESM_HIP(hipEventSynchronize(T.ev[2 * u + 1]));
    float ms = 0.f;
    SESM_HIP(hipEventElapsedTime(&ms, T.ev[2 * u], T.ev[2 * u + 1]));
    T.ms += ms;
  }
  T.used = 0;
  return SESM_OK;
}

int sesm_kt_begin(sesm_ctx* ctx, int id, hipStream_t st) {
  KTimer& T = ctx->kt[id];
  T.open = (T.calls++ % ctx->kt_every) == 0;
  if (!T.open) return SESM_OK;
  if (T.ev.empty()) {
    T.ev.assign(2 * SESM_KT_POOL, nullptr);
    for (hipEvent_t& e : T.ev) SESM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  if (T.used == SESM_KT_POOL) {
    const int rc = kt_fold(ctx, T);
    if (rc) return rc;
  }
  SESM_HIP(hipEventRecord(T.ev[2 * T.used], st));
  return SESM_OK;
}

int sesm_kt_end(sesm_ctx* ctx, int id, hipStream_t st, double nbytes) {
  KTimer& T = ctx->kt[id];
  if (!T.open) return SESM_OK;
  T.open = false;
  SESM_HIP(hipEventRecord(T.ev[2 * T.used + 1], st));
  ++T.used;
  ++T.launches;
  T.bytes += nbytes;
  return SESM_OK;
}

void sesm_kt_free(sesm_ctx* ctx) {
  for (KTimer& T : ctx->kt) {
    for (hipEvent_t e : T.ev)
      if (e) (void)hipEventDestroy(e);
    T = KTimer{};
  }
  ctx->kt_mask = 0;
}

int sesm_timing_enable(sesm_ctx* ctx, uint32_t mask, int32_t every) {
  if (!ctx) return SESM_EINVAL;
  if (mask >> SESM_KT_COUNT) return ctx->fail(SESM_EINVAL, "timing mask selects unknown kernel classes");
  if (every < 1) return ctx->fail(SESM_EINVAL, "timing sample interval must be >= 1");
  SESM_HIP(hipSetDevice(ctx->device));
  for (KTimer& T : ctx->kt) {
    const int rc = kt_fold(ctx, T);  // let recorded events finish before they are reused
    if (rc) return rc;
    T.launches = T.calls = 0;
    T.open = false;
    T.ms = T.bytes = 0.0;
  }
  ctx->kt_mask = mask;
  ctx->kt_every = every;
  return SESM_OK;
}

int sesm_timing_read(sesm_ctx* ctx, sesm_kernel_stat* stats, int32_t n_stats) {
  if (!ctx) return SESM_EINVAL;
  if (!stats || n_stats < SESM_KT_COUNT) return ctx->fail(SESM_EINVAL, "need SESM_KT_COUNT records");
  SESM_HIP(hipSetDevice(ctx->device));
  for (int i = 0; i < SESM_KT_COUNT; ++i) {
    KTimer& T = ctx->kt[i];
    const int rc = kt_fold(ctx, T);
    if (rc) return rc;
    sesm_kernel_stat& o = stats[i];
    std::memset(&o, 0, sizeof(o));
    std::strncpy(o.name, kKtNames[i], sizeof(o.name) - 1);
    o.launches = T.launches;
    o.total_ms = T.ms;
    o.bytes = T.bytes;
  }
  return SESM_OK;
}
