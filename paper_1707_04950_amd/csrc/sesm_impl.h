// Internal declarations of the sesm library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
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

// The incidence-dependent constants of the accelerated operator, one record
// per incidence (device memory): the Bloch phase e^{i alpha d} of wrapped
// columns and grid points (eq. shifted_periodic_green_function) and the
// completion modes of eq. M_eta.
struct IncParams {
  double alpha, alpha_d;
  int nU, pad;
  double Ua[SESM_MAX_UETA], Ubr[SESM_MAX_UETA], Ubi[SESM_MAX_UETA];
};

// Parameters handed by value to the operator kernels.
struct KParams {
  int N, j, n_a, pmin, pmax, nU;
  double d, k, alpha, dx, h, A_len, cA, a, gamma;
  double wshift[SESM_MAX_J + 1];
  double Ua[SESM_MAX_UETA], Ubr[SESM_MAX_UETA], Ubi[SESM_MAX_UETA];
};

struct AccelOp;  // shifted-equivalent-source accelerator (sesm_accel.hip)

// A near-field split chosen by the tuner for one accelerator grid shape.
struct NearSplit {
  int64_t key[8];
  int c1, c2, c3;
  double us;
};

// Event pairs of one timed kernel class (folded into ms when the pool is full
// and when read).
struct KTimer {
  std::vector<hipEvent_t> ev;  // 2 per launch slot
  int used = 0;                // recorded pairs not yet folded
  int64_t calls = 0;           // launches of the class since enabling
  int64_t launches = 0;        // launches timed
  bool open = false;           // the current launch is bracketed
  double ms = 0.0, bytes = 0.0;
};
#define SESM_KT_POOL 2048  // launch slots per class between folds

struct sesm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool ready = false;
  bool adjoint = false;  // dense-mode operator applications use the conjugate transpose (adjoint solves)
  Problem P;
  sesm_params prm{};
  // surface samples (device), length N
  double *x = nullptr, *f = nullptr, *fp = nullptr, *fpp = nullptr, *J = nullptr;
  double* logw = nullptr;  // log-quadrature weights R_m, m = 0..n_a-1
  cplx* Mdense = nullptr;  // dense operator, row-major N x N
  cplx* dA_dY = nullptr;   // with sesm_params.adjoint: dA/dY and dA/df' (row-major N x N each)
  cplx* dA_dF = nullptr;
  AccelOp* acc = nullptr;
  // GMRES workspace
  cplx* V = nullptr;
  int64_t V_cols = 0;
  cplx* hcol = nullptr;      // device Hessenberg columns (+ norm), a ring of SESM_HRING slots
  cplx* hpart = nullptr;     // partial dot products
  cplx* hhost = nullptr;     // pinned host ring slots of Hessenberg columns (+ one slot for uploads)
  cplx* hhost_dev = nullptr; // the same memory as the device sees it
  int64_t* hflag = nullptr;  // per ring slot: sequence number of the step whose column it holds
  int64_t* hflag_dev = nullptr;
  int64_t gm_seq = 0;        // steps enqueued on this context
  cplx* ybuf = nullptr;      // device copy of the small LS solution
  cplx* wtmp = nullptr;      // scratch vector of length N (the right-hand side when none is given)
  cplx* gw = nullptr;        // A u of the current Arnoldi step
  // mixed-precision solves: FP64 mirror of the current FP32 basis vector, the
  // inner solve's residual, the outer residual and correction (N each)
  cplx *umix = nullptr, *mx_r = nullptr, *mx_R = nullptr, *mx_D = nullptr;
  cplx* Hrow = nullptr;      // packed upper-Hessenberg matrix, row-major
  cplx* htri = nullptr;      // its columns gathered column-major (column j: rows 0..j+1)
  int64_t Hrow_len = 0;
  int Hrow_m = -1;
  cplx* hp = nullptr;        // first-pass coefficients of the newest column
  cplx* gcoef = nullptr;     // update coefficients (s, z, z - a s)
  double* gsc = nullptr;     // step scalars
  // host copies of the Hessenberg columns of a cycle, packed (column j: rows
  // 0..j+1 at j (j + 3) / 2), kept across solves so that their pages stay mapped
  std::vector<std::complex<double>> gm_rot, gm_raw;
  std::vector<cplx> gm_tri;
  // Rayleigh coefficients: per-order constants and results (device), room for
  // ray_cap orders; allocated with the surface
  void* ray_oc = nullptr;
  cplx* ray_B = nullptr;
  int ray_cap = 0;
  void* noalloc_scratch = nullptr;  // this device's copy of the library's fixed array (sesm_rayleigh_noalloc)
  std::vector<NearSplit> near_splits;  // tuned near-field splits by grid shape (kept across surfaces)
  std::vector<std::pair<void*, size_t>> owned;  // every device allocation made for the surface
  // device blocks released by an earlier surface, by size, reused by the next
  // one (a surface of the same shape allocates the same sizes); bounded below
  std::vector<std::pair<size_t, void*>> pool;
  size_t pool_bytes = 0;
  bool poison = false;       // fill new allocations with NaN bytes (SESM_POISON_ALLOC set at creation)
  int64_t bytes = 0;
  // per-kernel timing (sesm_timing_enable)
  uint32_t kt_mask = 0;
  int kt_every = 1;  // bracket every kt_every-th launch of a class
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
void sesm_pool_put(sesm_ctx* ctx, void* p, size_t bytes);  // hand a released device block to the pool

// dense path (sesm_dense.hip)
int sesm_dense_setup(sesm_ctx* ctx);
int sesm_dense_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y);

// accelerated path (sesm_accel.hip)
int sesm_accel_setup(sesm_ctx* ctx);
int sesm_accel_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y, bool mixed = false);
// inc0 < 0: every density with the surface's own incidence; inc0 >= 0: density
// r with member inc0 + r of the incidence set
// mixed: the mixed-precision map (EqSources operators in FP32)
int sesm_accel_matvec_batch(sesm_ctx* ctx, int nrhs, const cplx* mu, int64_t ldm, cplx* y, int64_t ldy,
                            int inc0 = -1, bool mixed = false);
int sesm_accel_set_incidences(sesm_ctx* ctx, int n, const double* alpha);
// Off-surface field (sesm_field): the accelerator's cell grid, and the field
// at the points inside it (point index idx[t], coordinates px[t], py[t] with
// px in [x0, x0 + d), quasi-periodic shift p[t] periods) into u (device, by
// point index), from one forward map of mu
struct AccelGrid {
  double x0, y0, L;
  int n_x, n_y;
};
AccelGrid sesm_accel_grid(const sesm_ctx* ctx);
int sesm_accel_field_cells(sesm_ctx* ctx, const cplx* mu, int n, const int* idx, const double* px, const double* py,
                           const int* p, cplx* u);
int sesm_accel_n_incidences(const sesm_ctx* ctx);
const Problem* sesm_accel_incidence(const sesm_ctx* ctx, int r);
void sesm_accel_free(sesm_ctx* ctx);
void sesm_accel_info(const sesm_ctx* ctx, sesm_surface_info* info);

// operator dispatch; sesm_apply_inc applies the operator of member inc of the
// incidence set (inc < 0: the surface's own incidence)
int sesm_apply(sesm_ctx* ctx, const cplx* mu, cplx* y);
int sesm_dense_assemble_with_derivs(sesm_ctx* ctx);
int sesm_dense_matvec_adjoint(sesm_ctx* ctx, const cplx* mu, cplx* y);
int sesm_apply_inc(sesm_ctx* ctx, const cplx* mu, cplx* y, int inc, bool mixed = false);

// incidence-dependent scalars (alpha, beta, U^eta, propagating orders) of P
bool sesm_problem_alpha(Problem& P, double alpha, double eta);

// dst[e] = src[e], e < n, by nt threads (tid = own index): B loads per thread
// are issued (indices clamped) before any store, so one memory latency covers
// B elements instead of each element waiting for its own load.
template <int B, typename T>
__device__ inline void stage_copy(T* dst, const T* __restrict__ src, int n, int tid, int nt) {
  for (int e0 = tid; e0 < n; e0 += B * nt) {
    T v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = src[min(e0 + u * nt, n - 1)];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (e0 + u * nt < n) dst[e0 + u * nt] = v[u];
  }
}

// Wavefront sums through DPP lane moves (no LDS traffic): quad permutes, row
// half-mirror and mirror give every lane its row's sum; row broadcasts of
// lanes 15 and 31 accumulate rows upward, so lane 63 holds the total, which
// readlane hands to every lane.  Each double moves as two 32-bit halves;
// lanes outside a broadcast's row mask receive 0.
template <int CTRL, int ROW_MASK>
__device__ inline double sesm_dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double wave_sum_d(double v) {
  v += sesm_dpp_mov<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += sesm_dpp_mov<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += sesm_dpp_mov<0x141, 0xF>(v);  // row_half_mirror
  v += sesm_dpp_mov<0x140, 0xF>(v);  // row_mirror
  v += sesm_dpp_mov<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += sesm_dpp_mov<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum over the wavefront, returned in every lane
__device__ inline cplx wave_sum(cplx v) { return cplx{wave_sum_d(v.re), wave_sum_d(v.im)}; }

// sums over aligned groups of G = 16, 32 or 64 lanes, valid in the last lane
// of each group
template <int G>
__device__ inline double group_sum_d(double v) {
  v += sesm_dpp_mov<0xB1, 0xF>(v);
  v += sesm_dpp_mov<0x4E, 0xF>(v);
  v += sesm_dpp_mov<0x141, 0xF>(v);
  v += sesm_dpp_mov<0x140, 0xF>(v);
  if (G >= 32) v += sesm_dpp_mov<0x142, 0xA>(v);
  if (G == 64) v += sesm_dpp_mov<0x143, 0xC>(v);
  return v;
}

// value of v in lane l (l wave-uniform), through the scalar unit
__device__ inline double sesm_readlane(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// block-level sum: wavefront sums, then LDS across wavefronts (NT multiple of 64)
template <int NT>
__device__ inline cplx block_sum(cplx v, cplx* sh) {
  v = wave_sum(v);
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
