// Internal declarations of the sesm library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sesm.h"
#include "sesm_math.h"

#define SESM_MAX_J 16
#define SESM_MAX_UETA 64
#define SESM_HRING 4       // Hessenberg column slots in flight
#define SESM_HSTRIDE 4208  // entries per slot (Krylov dimension <= 4000)

// Scalars of one discretised problem (Algorithm 2 inputs and derived sizes).
struct Problem {
  int N = 0, j = 0, n_a = 0, mode = SESM_MODE_DENSE;
  double d = 0, k = 0, alpha = 0, beta = 0, h = 0, A_len = 0, cA = 0, a = 0, gamma = 0, eta = 0, dx = 0;
  double wshift[SESM_MAX_J + 1];  // (-1)^m C(j,m), eq. (shifted_green_function)
  int pmin = 0, pmax = 0;         // image range of the windowed lattice sum
  int nU = 0;                     // |U^eta|
  int U[SESM_MAX_UETA];
  double Ua[SESM_MAX_UETA], Ubr[SESM_MAX_UETA], Ubi[SESM_MAX_UETA];  // alpha_n, beta_n
  int n_first = 0, n_count = 0;   // propagating orders
};

// Parameters handed by value to the operator kernels.
struct KParams {
  int N, j, n_a, pmin, pmax, nU;
  double d, k, alpha, dx, h, A_len, cA, a, gamma;
  double wshift[SESM_MAX_J + 1];
  double Ua[SESM_MAX_UETA], Ubr[SESM_MAX_UETA], Ubi[SESM_MAX_UETA];
};

struct AccelOp;  // shifted-equivalent-source accelerator (sesm_accel.hip)

// Event pairs of one timed kernel class (folded into ms when the pool is full
// and when read).
struct KTimer {
  std::vector<hipEvent_t> ev;  // 2 per launch slot
  int used = 0;                // recorded pairs not yet folded
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};
#define SESM_KT_POOL 2048  // launch slots per class between folds

struct sesm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool ready = false;
  Problem P;
  sesm_params prm{};
  // surface samples (device), length N
  double *x = nullptr, *f = nullptr, *fp = nullptr, *fpp = nullptr, *J = nullptr;
  double* logw = nullptr;  // log-quadrature weights R_m, m = 0..n_a-1
  cplx* Mdense = nullptr;  // dense operator, row-major N x N
  AccelOp* acc = nullptr;
  // GMRES workspace
  cplx* V = nullptr;
  int64_t V_cols = 0;
  cplx* hcol = nullptr;      // device Hessenberg columns (+ norm), a ring of SESM_HRING slots
  cplx* hpart = nullptr;     // partial dot products
  cplx* hhost = nullptr;     // pinned host copies of the ring slots (+ one slot for uploads)
  hipEvent_t hev[4] = {};    // per ring slot: its column has reached hhost
  cplx* ybuf = nullptr;      // device copy of the small LS solution
  cplx* wtmp = nullptr;      // scratch vector of length N (the right-hand side when none is given)
  cplx* gw = nullptr;        // A u of the current Arnoldi step
  cplx* upart = nullptr;     // partial sums of the Gram-Schmidt update
  cplx* Hrow = nullptr;      // packed upper-Hessenberg matrix, row-major
  int64_t Hrow_len = 0;
  int Hrow_m = -1;
  cplx* hp = nullptr;        // first-pass coefficients of the newest column
  cplx* gcoef = nullptr;     // update coefficients (s, z, z - a s)
  double* gsc = nullptr;     // step scalars
  std::vector<void*> owned;  // every device allocation made for the surface
  int64_t bytes = 0;
  // per-kernel timing (sesm_timing_enable)
  uint32_t kt_mask = 0;
  KTimer kt[SESM_KT_COUNT];

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  KParams kparams() const;
};

#define SESM_HIP(expr)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return ctx->fail(SESM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SESM_LAUNCH_CHECK()                                                                     \
  do {                                                                                          \
    hipError_t e_ = hipGetLastError();                                                          \
    if (e_ != hipSuccess) return ctx->fail(SESM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// timing brackets (no-ops unless the class is selected)
int sesm_kt_begin(sesm_ctx* ctx, int id, hipStream_t st);
int sesm_kt_end(sesm_ctx* ctx, int id, hipStream_t st, double bytes);
void sesm_kt_free(sesm_ctx* ctx);
#define SESM_KT_BEGIN(id, st)                                   \
  do {                                                          \
    if ((ctx->kt_mask >> (id)) & 1u) {                          \
      const int r_ = sesm_kt_begin(ctx, (id), (st));            \
      if (r_) return r_;                                        \
    }                                                           \
  } while (0)
#define SESM_KT_END(id, st, nbytes)                             \
  do {                                                          \
    if ((ctx->kt_mask >> (id)) & 1u) {                          \
      const int r_ = sesm_kt_end(ctx, (id), (st), (nbytes));    \
      if (r_) return r_;                                        \
    }                                                           \
  } while (0)

// allocation owned by the surface (freed by release_surface)
int sesm_alloc(sesm_ctx* ctx, void** p, size_t bytes);
void sesm_release_surface(sesm_ctx* ctx);

// dense path (sesm_dense.hip)
int sesm_dense_setup(sesm_ctx* ctx);
int sesm_dense_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y);

// accelerated path (sesm_accel.hip)
int sesm_accel_setup(sesm_ctx* ctx);
int sesm_accel_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y);
void sesm_accel_free(sesm_ctx* ctx);
void sesm_accel_info(const sesm_ctx* ctx, sesm_surface_info* info);

// operator dispatch
int sesm_apply(sesm_ctx* ctx, const cplx* mu, cplx* y);

// block-level reductions
template <int NT>
__device__ inline cplx block_sum(cplx v, cplx* sh) {
  // wave reduction then LDS across waves; NT multiple of 64
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o);
    v.im += __shfl_xor(v.im, o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  cplx r = cplx{0.0, 0.0};
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  }
  return r;  // valid in thread 0
}

__device__ inline cplx wave_sum(cplx v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o);
    v.im += __shfl_xor(v.im, o);
  }
  return v;
}
