// GMRES (Algorithm 1: "Run GMRES iterations, using the forward map").
//
// Arnoldi with classical Gram-Schmidt and delayed reorthogonalisation: the
// second Gram-Schmidt pass of a basis vector is carried out in the next
// Arnoldi step, together with the first pass of the next vector, so every
// step reads the Krylov basis twice (one dot-product sweep, one update sweep)
// instead of four times.  With Q = [q_0 .. q_{k-1}] orthonormal and u the
// new vector after one projection (A q_{k-1} = Q h + u), step k computes
//   w = A u;  s = Q^H u, rho = u^H u, z = Q^H w, zeta = u^H w   (one sweep)
//   beta = sqrt(rho - |s|^2);  column k-1 of H: (h + s, beta)
//   q_k = (u - Q s) / beta
//   c_k = (zeta - s^H z) / beta,  a = c_k / beta
//   u'  = (w - Q (z - a s) - a u) / beta = A q_k - [Q q_k] h'    (one sweep)
//   h'  = ([z; c_k] - H s) / beta   (first-pass coefficients of column k)
// which follows from A q_k = (w - A Q s) / beta and A Q = [Q q_k] H.  The
// initial residual enters as u in step 0 (Q empty), whose beta is its norm.
// The Hessenberg columns are rotated (Givens) on the host, which runs one
// Arnoldi step behind the device and receives each column through coherent
// pinned memory written by the step kernel.
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sesm_impl.h"

namespace {

constexpr int VB = 4;          // basis vectors per dot-product block
constexpr int NCHUNK = 240;    // N-chunks of the single-vector norm reduction
constexpr int DCHUNK = 16;     // N-chunks of the multi-vector dot products
constexpr int STEP_NT = 1024;  // threads of the one-block Arnoldi step

// Offset of row r of the packed upper-Hessenberg matrix (rows 0..m, row r
// holds columns max(0, r-1)..m-1 contiguously).
__host__ __device__ inline int64_t hrow_off(int r, int m) {
  if (r == 0) return 0;
  const int64_t t = r - 1;
  return m + t * (m + 1) - t * (t + 1) / 2;
}

// part[(v DCHUNK + c) 2 + 0] = sum_{i in chunk c} conj(V_v[i]) u[i],
// part[(v DCHUNK + c) 2 + 1] = sum_{i in chunk c} conj(V_v[i]) w[i] (w optional),
// v in [0, nv).  Loads are unconditional (vector index clamped, surplus terms
// masked) so that all basis loads of an iteration are in flight together.
// VT: storage of the basis (cplx; cplxf for the FP32 bases of mixed-precision
// solves); the sums are formed in FP64.
template <typename VT>
__device__ __forceinline__ void gm_dots(int N, int nv, const VT* __restrict__ V, int64_t ldv,
                                        const VT* __restrict__ u, const cplx* __restrict__ w,
                                        cplx* __restrict__ part) {
  __shared__ cplx sh[2][VB][4];
  const int c = blockIdx.x, v0 = blockIdx.y * VB;
  const int per = (N + DCHUNK - 1) / DCHUNK;
  const int lo = c * per, hi = min(N, lo + per);
  const bool has_w = w != nullptr;
  const VT* row[VB];
  double msk[VB];
#pragma unroll
  for (int t = 0; t < VB; ++t) {
    row[t] = V + (int64_t)min(v0 + t, nv - 1) * ldv;
    msk[t] = v0 + t < nv ? 1.0 : 0.0;
  }
  cplx au[VB], aw[VB];
#pragma unroll
  for (int t = 0; t < VB; ++t) au[t] = aw[t] = cplx{0.0, 0.0};
  // software pipelined: the loads of element i + 256 are issued before the
  // products of element i
  int i = lo + threadIdx.x;
  cplx a[VB], ui = cplx{0.0, 0.0}, wi = cplx{0.0, 0.0};
  if (i < hi) {
#pragma unroll
    for (int t = 0; t < VB; ++t) a[t] = widen(row[t][i]);
    ui = widen(u[i]);
    wi = has_w ? w[i] : cplx{0.0, 0.0};
  }
  for (; i < hi; i += 256) {
    const int in = i + 256 < hi ? i + 256 : i;
    cplx b[VB];
#pragma unroll
    for (int t = 0; t < VB; ++t) b[t] = widen(row[t][in]);
    const cplx un = widen(u[in]);
    const cplx wn = has_w ? w[in] : cplx{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < VB; ++t) {
      au[t] = cmac_conj(au[t], a[t], ui);
      aw[t] = cmac_conj(aw[t], a[t], wi);
    }
#pragma unroll
    for (int t = 0; t < VB; ++t) a[t] = b[t];
    ui = un;
    wi = wn;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < VB; ++t) {
    const cplx s0 = wave_sum(au[t]);
    const cplx s1 = wave_sum(aw[t]);
    if (lane == 0) {
      sh[0][t][wv] = msk[t] * s0;
      sh[1][t][wv] = msk[t] * s1;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * VB) {
    const int t = threadIdx.x >> 1, j = threadIdx.x & 1;
    if (v0 + t < nv)
      part[((int64_t)(v0 + t) * DCHUNK + c) * 2 + j] = sh[j][t][0] + sh[j][t][1] + sh[j][t][2] + sh[j][t][3];
  }
}

// Arnoldi step k (one workgroup): reduce the dot products of k_gm_dots over
// V_0..V_k (V_k = u), then beta, the final column k-1 (hp + s, beta) into the
// packed Hessenberg matrix and contiguously into hout (device; for k = 0,
// hout[0] = beta, the residual norm), and the update coefficients
// cS = s, cZ = z, cC = z - a s; sc = (1/beta, Re a, Im a, beta, Re c_k, Im c_k).
// beta = 0 (an invariant Krylov space) gives zero coefficients and 1/beta = 0.
// The column reaches the host from the last workgroup of the update launch
// (or of k_gm_publish when no update follows).
__device__ __forceinline__ void gm_step(int k, int m, const cplx* __restrict__ part, const cplx* __restrict__ hp,
                                        cplx* __restrict__ Hrow, cplx* __restrict__ hout, cplx* __restrict__ cS,
                                        cplx* __restrict__ cZ, cplx* __restrict__ cC, double* __restrict__ sc) {
  constexpr int STEP_LDS = 2048, PER = (SESM_HSTRIDE + STEP_NT - 1) / STEP_NT;
  __shared__ cplx sh[STEP_NT / 64];
  __shared__ cplx s_last[2];  // (rho, zeta)
  __shared__ double s_beta;
  __shared__ cplx s_a;
  __shared__ cplx lS[STEP_LDS], lZ[STEP_LDS];  // s and z of the first STEP_LDS vectors
  // this thread's first-pass coefficients, loaded while the partials are reduced
  cplx hpv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int v = threadIdx.x + j * STEP_NT;
    hpv[j] = v < k ? hp[v] : cplx{0.0, 0.0};
  }
  // reduce the partials: lane = 16 g + c takes chunk c of basis vector
  // vb + 4 u + g (u < 4), so each wavefront has 16 vectors' loads in flight;
  // sums over the 16 chunks (DPP group sums, valid in lane c = 15) against u go
  // to cS, against w to cZ (v = k: rho and zeta)
  static_assert(DCHUNK == 16, "lane layout assumes 16 chunks");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  constexpr int U = 4;
  for (int vb = wv * 4 * U; vb <= k; vb += (STEP_NT / 64) * 4 * U) {
    cplx p0[U], p1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = min(vb + 4 * u + g, k);
      p0[u] = part[((int64_t)v * DCHUNK + c) * 2];
      p1[u] = part[((int64_t)v * DCHUNK + c) * 2 + 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = vb + 4 * u + g;
      const cplx s0 = cplx{group_sum_d<16>(p0[u].re), group_sum_d<16>(p0[u].im)};
      const cplx s1 = cplx{group_sum_d<16>(p1[u].re), group_sum_d<16>(p1[u].im)};
      if (c == 15 && v <= k) {
        if (v < k) {
          cS[v] = s0;
          cZ[v] = s1;
          if (v < STEP_LDS) {
            lS[v] = s0;
            lZ[v] = s1;
          }
        } else {
          s_last[0] = s0;
          s_last[1] = s1;
        }
      }
    }
  }
  __syncthreads();
  double ns = 0.0;
  cplx sz = cplx{0.0, 0.0};
  for (int v = threadIdx.x; v < k; v += STEP_NT) {
    const cplx av = v < STEP_LDS ? lS[v] : cS[v], bv = v < STEP_LDS ? lZ[v] : cZ[v];
    ns += abs2(av);
    sz += cmul_conj(av, bv);
  }
  const cplx t_ns = block_sum<STEP_NT>(cplx{ns, 0.0}, sh);
  const cplx t_sz = block_sum<STEP_NT>(sz, sh);
  if (threadIdx.x == 0) {
    const double b2 = s_last[0].re - t_ns.re;
    const double beta = b2 > 0.0 ? sqrt(b2) : 0.0;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    const cplx ck = inv * (s_last[1] - t_sz);
    const cplx a = inv * ck;
    s_beta = beta;
    s_a = a;
    sc[0] = inv;
    sc[1] = a.re;
    sc[2] = a.im;
    sc[3] = beta;
    sc[4] = ck.re;
    sc[5] = ck.im;
    if (k == 0) hout[0] = cplx{beta, 0.0};
  }
  __syncthreads();
  const cplx a = s_a;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int v = threadIdx.x + j * STEP_NT;
    if (v < k) {
      const cplx av = v < STEP_LDS ? lS[v] : cS[v], bv = v < STEP_LDS ? lZ[v] : cZ[v];
      cC[v] = bv - a * av;
      const cplx hv = hpv[j] + av;
      hout[v] = hv;
      Hrow[hrow_off(v, m) + (k - 1 - (v > 0 ? v - 1 : 0))] = hv;
    }
  }
  if (threadIdx.x == 0 && k > 0) {
    hout[k] = cplx{s_beta, 0.0};
    Hrow[hrow_off(k, m)] = cplx{s_beta, 0.0};
  }
}

// Copies the step's column (device, k + 1 entries) to its host ring slot,
// then, once every writer has released its entries at system scope and the
// workgroup has met, stores seq into *flag, which the host polls.
__device__ inline void gm_publish(int n, const cplx* __restrict__ col, cplx* __restrict__ hout, int64_t* flag,
                                  int64_t seq) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) hout[t] = col[t];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    flag[0] = seq;  // (vector store from one lane)
  }
}

__global__ __launch_bounds__(256) void k_gm_publish(int n, const cplx* __restrict__ col, cplx* __restrict__ hout,
                                                    int64_t* flag, int64_t seq) {
  gm_publish(n, col, hout, flag, seq);
}

// Second sweep of step k, with the first-pass coefficients of column k.
// Workgroups [0, nrb): rows 64 rb .. 64 rb + 63, one row per lane; wavefront
// g takes the basis vectors v = g, g + 4, ... < k, so the sums
// Q s = sum_v V_v cS[v] and Q cC = sum_v V_v cC[v] need no exchange between
// workgroups; the four wavefronts' sums are added through LDS and the
// workgroup forms
//   q_k = (u - Q s) / beta into V_k (in place of u),
//   u'  = (w - Q cC - a u) / beta into V_{k+1}.
// The following ceil((k+1)/4) workgroups compute the first-pass coefficients
// of column k, one wavefront per row r:
// hp[r] = (c_r - sum_{j >= max(0, r-1)} H[r][j] cS[j]) / beta, c = (cZ, c_k).
// With an FP32 basis (VT = cplxf) the new vectors are stored rounded and
// unext (when given) receives u' as stored, widened to FP64: the input of
// the next forward map, so that the Arnoldi relation holds for the stored basis.
constexpr int UPD_ROWS = 64, UPD_B = 8;
template <typename VT>
__device__ __forceinline__ void gm_update(int N, int k, int m, int nrb, VT* V, int64_t ldv,
                                          const cplx* __restrict__ cS, const cplx* __restrict__ cZ,
                                          const cplx* __restrict__ cC, const double* __restrict__ sc,
                                          const cplx* __restrict__ Hrow, cplx* __restrict__ hp,
                                          const cplx* __restrict__ w, const cplx* __restrict__ col,
                                          cplx* __restrict__ hout, int64_t* flag, int64_t seq,
                                          cplx* __restrict__ unext) {
  const int bid = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (bid == (int)gridDim.x - 1) {  // the last workgroup hands the step's column to the host
    gm_publish(k + 1, col, hout, flag, seq);
    return;
  }
  if (bid >= nrb) {
    const int r = (bid - nrb) * 4 + wv;
    if (r > k) return;  // wave-uniform
    const int j0 = r > 0 ? r - 1 : 0;
    const cplx* hr = Hrow + hrow_off(r, m) - j0;
    cplx acc = cplx{0.0, 0.0};
#pragma unroll 4
    for (int j = j0 + lane; j < k; j += 64) acc += hr[j] * cS[j];
    acc = wave_sum(acc);
    if (lane == 0) {
      const cplx cr = r < k ? cZ[r] : cplx{sc[4], sc[5]};
      hp[r] = sc[0] * (cr - acc);
    }
    return;
  }
  __shared__ cplx red[2][4][UPD_ROWS];
  const int i = min(bid * UPD_ROWS + lane, N - 1);  // rows past N repeat row N-1 (not stored)
  cplx s1 = cplx{0.0, 0.0}, s2 = cplx{0.0, 0.0};
  int v = wv;
  for (; v + 4 * (UPD_B - 1) < k; v += 4 * UPD_B) {  // UPD_B vectors' loads in flight
    cplx x[UPD_B], a1[UPD_B], a2[UPD_B];
#pragma unroll
    for (int t = 0; t < UPD_B; ++t) {
      x[t] = widen(V[(int64_t)(v + 4 * t) * ldv + i]);
      a1[t] = cS[v + 4 * t];
      a2[t] = cC[v + 4 * t];
    }
#pragma unroll
    for (int t = 0; t < UPD_B; ++t) {
      s1 = cmac(s1, x[t], a1[t]);
      s2 = cmac(s2, x[t], a2[t]);
    }
  }
  // (the remaining vectors one at a time: a tail padded with zero-weight
  // loads measured slower)
  for (; v < k; v += 4) {
    const cplx x = widen(V[(int64_t)v * ldv + i]);
    s1 = cmac(s1, x, cS[v]);
    s2 = cmac(s2, x, cC[v]);
  }
  red[0][wv][lane] = s1;
  red[1][wv][lane] = s2;
  __syncthreads();
  if (wv == 0 && bid * UPD_ROWS + lane < N) {
    const cplx p1 = red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
    const cplx p2 = red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane];
    const double inv = sc[0];
    const cplx a = cplx{sc[1], sc[2]};
    const cplx u = widen(V[(int64_t)k * ldv + i]);
    V[(int64_t)k * ldv + i] = narrow_to<VT>(inv * (u - p1));
    const VT un = narrow_to<VT>(inv * (w[i] - p2 - a * u));
    V[(int64_t)(k + 1) * ldv + i] = un;
    if (unext) unext[i] = widen(un);
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_gm_dots(int N, int nv, const VT* __restrict__ V, int64_t ldv,
                                                 const VT* __restrict__ u, const cplx* __restrict__ w,
                                                 cplx* __restrict__ part) {
  gm_dots<VT>(N, nv, V, ldv, u, w, part);
}
__global__ __launch_bounds__(STEP_NT) void k_gm_step(int k, int m, const cplx* __restrict__ part,
                                                     const cplx* __restrict__ hp, cplx* __restrict__ Hrow,
                                                     cplx* __restrict__ hout, cplx* __restrict__ cS,
                                                     cplx* __restrict__ cZ, cplx* __restrict__ cC,
                                                     double* __restrict__ sc) {
  gm_step(k, m, part, hp, Hrow, hout, cS, cZ, cC, sc);
}
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_update(int N, int k, int m, int nrb, VT* V, int64_t ldv,
                                                   const cplx* __restrict__ cS, const cplx* __restrict__ cZ,
                                                   const cplx* __restrict__ cC, const double* __restrict__ sc,
                                                   const cplx* __restrict__ Hrow, cplx* __restrict__ hp,
                                                   const cplx* __restrict__ w, const cplx* __restrict__ col,
                                                   cplx* __restrict__ hout, int64_t* flag, int64_t seq,
                                                   cplx* __restrict__ unext) {
  gm_update<VT>(N, k, m, nrb, V, ldv, cS, cZ, cC, sc, Hrow, hp, w, col, hout, flag, seq, unext);
}

// The systems of a batched solve: member q's buffers are the base pointers
// plus q times the strides (bases (m + 1) x N, A u, the small per-member
// buffers, the device view of its pinned ring slots and flags).  The active
// members are the set bits of `active`; the i-th of them runs with sequence
// number seq0 + i.
struct GmBatch {
  void* V;           // bases, stored as cplx or cplxf (the kernels' VT)
  int64_t vstride;
  cplx* U;           // FP32 bases: each member's next forward-map input (N each), else null
  cplx* W;
  cplx* small;
  int64_t sstride, o_hcol, o_hpart, o_hp, o_gcoef, o_gsc, o_Hrow;
  cplx* pin;
  int64_t pstride;
  int64_t seq0;
  uint64_t active;
};

// index of the i-th set bit of mask (i < popcount(mask))
__device__ inline int gm_nth_member(uint64_t mask, int i) {
  for (int t = 0; t < i; ++t) mask &= mask - 1;
  return __builtin_ctzll(mask);
}

// Arnoldi step k of every active member (grid dimension z for the sweeps,
// x for the one-workgroup step): the same bodies as the single-system
// kernels, on the member's buffers.
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_dots_batch(GmBatch B, int N, int k, int full) {
  const int q = gm_nth_member(B.active, blockIdx.z);
  const VT* V = static_cast<const VT*>(B.V) + q * B.vstride;
  cplx* sm = B.small + q * B.sstride;
  gm_dots<VT>(N, k + 1, V, N, V + (int64_t)k * N, full ? B.W + (int64_t)q * N : nullptr, sm + B.o_hpart);
}
__global__ __launch_bounds__(STEP_NT) void k_gm_step_batch(GmBatch B, int k, int m) {
  const int q = gm_nth_member(B.active, blockIdx.x);
  cplx* sm = B.small + q * B.sstride;
  cplx* cS = sm + B.o_gcoef;
  gm_step(k, m, sm + B.o_hpart, sm + B.o_hp, sm + B.o_Hrow, sm + B.o_hcol + (int64_t)(k % 2) * SESM_HSTRIDE, cS,
          cS + SESM_HSTRIDE, cS + 2 * SESM_HSTRIDE, reinterpret_cast<double*>(sm + B.o_gsc));
}
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_update_batch(GmBatch B, int N, int k, int m, int nrb) {
  const int i = blockIdx.z, q = gm_nth_member(B.active, i);
  VT* V = static_cast<VT*>(B.V) + q * B.vstride;
  cplx* sm = B.small + q * B.sstride;
  const cplx* cS = sm + B.o_gcoef;
  cplx* ring = B.pin + q * B.pstride;
  const int slot = k % SESM_HRING;
  int64_t* flags = reinterpret_cast<int64_t*>(ring + (int64_t)(SESM_HRING + 1) * SESM_HSTRIDE);
  gm_update(N, k, m, nrb, V, N, cS, cS + SESM_HSTRIDE, cS + 2 * SESM_HSTRIDE, reinterpret_cast<const double*>(sm + B.o_gsc),
            sm + B.o_Hrow, sm + B.o_hp, B.W + (int64_t)q * N, sm + B.o_hcol + (int64_t)(k % 2) * SESM_HSTRIDE,
            ring + (int64_t)slot * SESM_HSTRIDE, flags + slot, B.seq0 + i, B.U ? B.U + (int64_t)q * N : nullptr);
}
// the last step of a cycle (no update follows): each member publishes its column
__global__ __launch_bounds__(256) void k_gm_publish_batch(GmBatch B, int k) {
  const int i = blockIdx.x, q = gm_nth_member(B.active, i);
  cplx* sm = B.small + q * B.sstride;
  cplx* ring = B.pin + q * B.pstride;
  const int slot = k % SESM_HRING;
  int64_t* flags = reinterpret_cast<int64_t*>(ring + (int64_t)(SESM_HRING + 1) * SESM_HSTRIDE);
  gm_publish(k + 1, sm + B.o_hcol + (int64_t)(k % 2) * SESM_HSTRIDE, ring + (int64_t)slot * SESM_HSTRIDE,
             flags + slot, B.seq0 + i);
}

// Columns 0..nv-1 of the packed Hessenberg matrix, column-major: column j
// (rows 0..j+1) at tri[j (j + 3) / 2 ..], one workgroup per column.
__global__ __launch_bounds__(256) void k_hess_gather(int m, const cplx* __restrict__ Hrow, cplx* __restrict__ tri) {
  const int j = blockIdx.x;
  for (int r = threadIdx.x; r <= j + 1; r += 256)
    tri[(int64_t)j * (j + 3) / 2 + r] = Hrow[hrow_off(r, m) + (j - (r > 0 ? r - 1 : 0))];
}

// x[i] += sum_{v < nv} V_v[i] y[v]
template <typename VT>
__global__ __launch_bounds__(256) void k_combine(int N, int nv, const VT* __restrict__ V, int64_t ldv,
                                                 const cplx* __restrict__ y, cplx* __restrict__ x) {
  extern __shared__ cplx ys[];
  for (int v = threadIdx.x; v < nv; v += 256) ys[v] = y[v];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  cplx s = x[i];
  for (int v = 0; v < nv; ++v) s += widen(V[(int64_t)v * ldv + i]) * ys[v];
  x[i] = s;
}

// The first basis vector from r: V0 = r as stored (VT) and, for an FP32
// basis, u0 = that value widened (the first forward-map input).
template <typename VT>
__global__ void k_basis0(int N, const cplx* __restrict__ r, VT* __restrict__ V0, cplx* __restrict__ u0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const VT v = narrow_to<VT>(r[i]);
  V0[i] = v;
  if (u0) u0[i] = widen(v);
}

// x += d; r = b - r (a forward map's output in r)
__global__ void k_axpy1(int N, cplx* __restrict__ x, const cplx* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) x[i] = x[i] + d[i];
}

__global__ __launch_bounds__(256) void k_norm2_part(int N, const cplx* __restrict__ w, double* __restrict__ part) {
  __shared__ cplx sh[4];
  const int per = (N + NCHUNK - 1) / NCHUNK;
  const int lo = blockIdx.x * per, hi = min(N, lo + per);
  double s = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += 256) s += abs2(w[i]);
  const cplx r = block_sum<256>(cplx{s, 0.0}, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r.re;
}

// out = cplx(sqrt(sum part), 0)
__global__ void k_norm_final(const double* __restrict__ part, cplx* __restrict__ out) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int c = lane; c < NCHUNK; c += 64) s += part[c];
  s = wave_sum(cplx{s, 0.0}).re;
  if (lane == 0) *out = cplx{sqrt(s), 0.0};
}

// r = b - r
__global__ void k_sub_from(int N, const cplx* __restrict__ b, cplx* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  r[i] = b[i] - r[i];
}

// A signalling-NaN bit pattern that no arithmetic produces (results are
// quiet NaNs at worst): every entry of a host ring slot holds it until the
// step kernel's value has arrived, and again after the host has taken it.
constexpr uint64_t kColumnSentinel = 0x7FF4A5A5A5A5A5A5ull;
inline double column_sentinel() {
  double v;
  std::memcpy(&v, &kColumnSentinel, sizeof v);
  return v;
}
inline bool is_column_sentinel(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof b);
  return b == kColumnSentinel;
}

// entries of the gathered columns 0..m-1 (column j holds j + 2)
inline int64_t m_tri(int m) { return m > 0 ? (int64_t)m * (m + 3) / 2 : 0; }

// The small per-context buffers of a solve (Hessenberg column ring, partial
// sums, step scalars, work vectors of N) and the pinned host slots; kept
// until the surface is released.
int ensure_small(sesm_ctx* ctx) {
  const int N = ctx->P.N;
  int rc;
  if (!ctx->hcol) {
    if ((rc = sesm_alloc(ctx, (void**)&ctx->hcol, sizeof(cplx) * SESM_HRING * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->hpart, sizeof(cplx) * (size_t)2 * SESM_HSTRIDE * DCHUNK))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->ybuf, sizeof(cplx) * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->hp, sizeof(cplx) * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->gcoef, sizeof(cplx) * 3 * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->gsc, sizeof(double) * 8))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->wtmp, sizeof(cplx) * (size_t)N))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->gw, sizeof(cplx) * (size_t)N))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->umix, sizeof(cplx) * (size_t)N)) ||
        (rc = sesm_alloc(ctx, (void**)&ctx->mx_r, sizeof(cplx) * (size_t)N)) ||
        (rc = sesm_alloc(ctx, (void**)&ctx->mx_R, sizeof(cplx) * (size_t)N)) ||
        (rc = sesm_alloc(ctx, (void**)&ctx->mx_D, sizeof(cplx) * (size_t)N)))
      return rc;
  }
  if (!ctx->hhost || !ctx->hflag) {
    // columns and their flags in coherent pinned memory, written by the update
    // launch (kept for the context's lifetime)
    if (ctx->hhost) (void)hipHostFree(ctx->hhost);
    if (ctx->hflag) (void)hipHostFree(ctx->hflag);
    ctx->hhost = nullptr;
    ctx->hflag = nullptr;
    if (hipHostMalloc((void**)&ctx->hhost, sizeof(cplx) * (SESM_HRING + 1) * SESM_HSTRIDE, hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void**)&ctx->hflag, sizeof(int64_t) * SESM_HRING, hipHostMallocCoherent) != hipSuccess)
      return ctx->fail(SESM_ENOMEM, "hipHostMalloc failed");
    for (int t = 0; t < SESM_HRING; ++t) ctx->hflag[t] = 0;
    double* hv = reinterpret_cast<double*>(ctx->hhost);
    for (size_t t = 0; t < (size_t)2 * SESM_HRING * SESM_HSTRIDE; ++t) hv[t] = column_sentinel();
    SESM_HIP(hipHostGetDevicePointer((void**)&ctx->hhost_dev, ctx->hhost, 0));
    SESM_HIP(hipHostGetDevicePointer((void**)&ctx->hflag_dev, ctx->hflag, 0));
  }
  return SESM_OK;
}

int ensure_workspace(sesm_ctx* ctx, int m) {
  const int N = ctx->P.N;
  if (ctx->V && ctx->V_cols >= m + 1 && ctx->Hrow_m == m) return SESM_OK;
  auto drop = [&](void* p) {
    if (!p) return;
    for (size_t t = 0; t < ctx->owned.size(); ++t)
      if (ctx->owned[t].first == p) {
        sesm_pool_put(ctx, p, ctx->owned[t].second);
        ctx->owned.erase(ctx->owned.begin() + t);
        break;
      }
  };
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->V) ctx->bytes -= (int64_t)ctx->V_cols * N * (int64_t)sizeof(cplx);
  if (ctx->Hrow) ctx->bytes -= ctx->Hrow_len * (int64_t)sizeof(cplx);
  if (ctx->htri) ctx->bytes -= (int64_t)m_tri(ctx->Hrow_m) * (int64_t)sizeof(cplx);
  drop(ctx->V);
  drop(ctx->Hrow);
  drop(ctx->htri);
  ctx->V = ctx->Hrow = ctx->htri = nullptr;
  ctx->V_cols = ctx->Hrow_len = 0;
  ctx->Hrow_m = -1;
  int rc = sesm_alloc(ctx, (void**)&ctx->V, sizeof(cplx) * (size_t)(m + 1) * N);
  if (rc) return rc;
  ctx->V_cols = m + 1;
  ctx->Hrow_len = hrow_off(m, m) + 1;
  if ((rc = sesm_alloc(ctx, (void**)&ctx->Hrow, sizeof(cplx) * (size_t)ctx->Hrow_len))) return rc;
  if ((rc = sesm_alloc(ctx, (void**)&ctx->htri, sizeof(cplx) * (size_t)m_tri(m)))) return rc;
  ctx->Hrow_m = m;
  if ((rc = ensure_small(ctx))) return rc;
  return SESM_OK;
}

using Cd = std::complex<double>;

// plain complex product (no special-value handling: the operands are finite)
inline Cd gm_mul(Cd a, Cd b) {
  return Cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

// Givens QR of one Hessenberg column j (rows 0..j+1, in place) given the
// rotations of the columns before it; updates g and returns |g[j+1]|
double gm_rotate(Cd* col, int j, std::vector<Cd>& cs, std::vector<Cd>& sn, std::vector<Cd>& g) {
  for (int t = 0; t < j; ++t) {  // previous rotations [[conj c, conj s], [-s, c]]
    const Cd p = col[t], q = col[t + 1];
    col[t] = gm_mul(std::conj(cs[t]), p) + gm_mul(std::conj(sn[t]), q);
    col[t + 1] = gm_mul(cs[t], q) - gm_mul(sn[t], p);
  }
  const Cd a = col[j], bb = col[j + 1];
  const double r = std::sqrt(std::norm(a) + std::norm(bb));
  cs[j] = r != 0 ? a / r : 1.0;
  sn[j] = r != 0 ? bb / r : 0.0;
  col[j] = r;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = std::conj(cs[j]) * g[j];
  return std::abs(g[j + 1]);
}

// wait until a step's column has reached the host (its flag carries the
// step's sequence number); fall back to a stream synchronisation after 2 s
int gm_wait(sesm_ctx* ctx, volatile int64_t* fl, int64_t seq) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int spin = 0; *fl != seq; ++spin) {
    if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      SESM_HIP(hipStreamSynchronize(ctx->stream));
      if (*fl != seq) return ctx->fail(SESM_EHIP, "GMRES step result did not reach the host");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return SESM_OK;
}

// After the flag, take the n entries of a host slot once none holds the
// sentinel any more (an entry's store may reach host memory after the
// flag's), then put the sentinel back.  Falls back to a stream
// synchronisation after 2 s.
int gm_take(sesm_ctx* ctx, cplx* slot_mem, int n, Cd* dst) {
  volatile double* hv = reinterpret_cast<volatile double*>(slot_mem);
  const auto t0 = std::chrono::steady_clock::now();
  for (int spin = 0;; ++spin) {
    int t = 0;
    while (t < 2 * n && !is_column_sentinel(hv[t])) ++t;
    if (t == 2 * n) break;
    if ((spin & 255) == 255 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      SESM_HIP(hipStreamSynchronize(ctx->stream));
      for (t = 0; t < 2 * n; ++t)
        if (is_column_sentinel(hv[t])) return ctx->fail(SESM_EHIP, "GMRES column did not reach the host");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  for (int t = 0; t < n; ++t) dst[t] = Cd(hv[2 * t], hv[2 * t + 1]);
  for (int t = 0; t < 2 * n; ++t) hv[t] = column_sentinel();
  return SESM_OK;
}

}  // namespace

// ||r|| / bnorm for a device vector r (norm partials and the result through the
// context's small buffers and the host upload slot; synchronises the stream)
static int gm_rel_norm(sesm_ctx* ctx, const cplx* r, double bnorm, double* out) {
  hipStream_t st = ctx->stream;
  const int N = ctx->P.N;
  hipLaunchKernelGGL(k_norm2_part, dim3(NCHUNK), dim3(256), 0, st, N, r, (double*)ctx->hpart);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, (const double*)ctx->hpart, ctx->hcol);
  SESM_LAUNCH_CHECK();
  cplx* hup = ctx->hhost + (size_t)SESM_HRING * SESM_HSTRIDE;
  SESM_HIP(hipMemcpyAsync(hup, ctx->hcol, sizeof(cplx), hipMemcpyDeviceToHost, st));
  SESM_HIP(hipStreamSynchronize(st));
  *out = bnorm > 0.0 ? hup[0].re / bnorm : hup[0].re;
  return SESM_OK;
}

// r = b - A x (one forward map; the operator of incidence inc, or the
// surface's own when inc < 0; mixed: the mixed-precision map)
static int gm_residual(sesm_ctx* ctx, const cplx* b, const cplx* x, cplx* r, int inc, bool mixed = false) {
  const int rc = sesm_apply_inc(ctx, x, r, inc, mixed);
  if (rc) return rc;
  const int N = ctx->P.N;
  hipLaunchKernelGGL(k_sub_from, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, b, r);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

// The single-system solve.  prev_true: the true relative residual of the
// initial guess when the caller has already formed it (a batched solve
// continuing one of its systems), else infinity; a restart from the true
// residual must at least halve it, otherwise the forward map's rounding floor
// has been reached and the solve stops.
// inc >= 0: the operator and incident field of member inc of the incidence set.
// VT: storage of the Krylov basis.  With VT = cplxf (the inner solves of a
// mixed-precision solve) the forward map is the mixed-precision one when
// mixed is set, and its input is the FP64 mirror ctx->umix of the current
// basis vector.
template <typename VT>
static int solve_impl_t(sesm_ctx* ctx, const sesm_c64* b_in, sesm_c64* mu_out, double tol, int32_t max_iter,
                        int32_t restart, int32_t flags, double prev_true, sesm_solve_info* info, int inc, bool mixed) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu_out || !(tol > 0) || max_iter < 1 || max_iter > 100000 || restart < 0 || (flags & ~SESM_SOLVE_X0))
    return ctx->fail(SESM_EINVAL, "bad solve arguments");
  if (b_in && (const void*)b_in == (const void*)mu_out) return ctx->fail(SESM_EINVAL, "b and mu must differ");
  SESM_HIP(hipSetDevice(ctx->device));
  const int N = ctx->P.N;
  const int m = (restart == 0 || restart > max_iter) ? max_iter : restart;
  if (m > 4000) return ctx->fail(SESM_EINVAL, "Krylov dimension above 4000; use restart");
  int rc = ensure_workspace(ctx, m);
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  const int nb = (N + 255) / 256;
  cplx* x = (cplx*)mu_out;
  VT* V = reinterpret_cast<VT*>(ctx->V);  // (the allocation holds (m + 1) N complex FP64 values)
  const int64_t ldv = N;
  constexpr bool f32 = !std::is_same<VT, cplx>::value;
  cplx* um = f32 ? ctx->umix : nullptr;                           // FP64 mirror of the current basis vector
  cplx* rb = f32 ? ctx->mx_r : reinterpret_cast<cplx*>(V);       // where the residual is formed (V_0 itself for FP64)
  cplx* cS = ctx->gcoef;
  cplx* cZ = cS + SESM_HSTRIDE;
  cplx* cC = cZ + SESM_HSTRIDE;
  const bool warm = (flags & SESM_SOLVE_X0) != 0;

  // right-hand side (incident field written into the workspace vector when NULL)
  const cplx* b = (const cplx*)b_in;
  if (!b) {
    if ((rc = inc < 0 ? sesm_rhs(ctx, (sesm_c64*)ctx->wtmp) : sesm_rhs_incidence(ctx, inc, (sesm_c64*)ctx->wtmp)))
      return rc;
    b = ctx->wtmp;
  }
  double bnorm = 0.0;
  if ((rc = gm_rel_norm(ctx, b, 0.0, &bnorm))) return rc;
  cplx* hup = ctx->hhost + (size_t)SESM_HRING * SESM_HSTRIDE;  // the host slot for small transfers
  if (!warm || bnorm == 0.0) SESM_HIP(hipMemsetAsync(x, 0, sizeof(cplx) * (size_t)N, st));
  sesm_solve_info inf{};
  if (bnorm == 0.0) {  // the solution of A x = 0 is x = 0
    SESM_HIP(hipStreamSynchronize(st));
    inf.converged = 1;
    if (info) *info = inf;
    return SESM_OK;
  }

  int64_t slot_seq[SESM_HRING] = {};
  // Arnoldi step k of a cycle with `steps` columns: steps k < steps apply the
  // operator and update the basis; step `steps` only finalises the last
  // column.  The step's column (for k = 0: the residual norm) goes to ring
  // slot k % SESM_HRING and then to the host.
  auto arnoldi = [&](int k, int steps) -> int {
    const bool full = k < steps;
    VT* u = V + (int64_t)k * ldv;
    if (full) {
      const int r = sesm_apply_inc(ctx, f32 ? um : reinterpret_cast<const cplx*>(u), ctx->gw, inc, mixed);
      if (r) return r;
    }
    const int nv = k + 1, slot = k % SESM_HRING;
    const double c16 = sizeof(VT);
    SESM_KT_BEGIN(SESM_KT_DOTS, st);
    hipLaunchKernelGGL(k_gm_dots<VT>, dim3(DCHUNK, (nv + VB - 1) / VB), dim3(256), 0, st, N, nv, V, ldv, u,
                       full ? ctx->gw : nullptr, ctx->hpart);
    SESM_LAUNCH_CHECK();
    // basis (u among it), w, partials
    SESM_KT_END(SESM_KT_DOTS, st, c16 * ((double)nv * N + (full ? N : 0) + 2.0 * nv * DCHUNK));
    const int64_t seq = ++ctx->gm_seq;
    cplx* colv = ctx->hcol + (size_t)(k % 2) * SESM_HSTRIDE;  // the step's column on the device
    hipLaunchKernelGGL(k_gm_step, dim3(1), dim3(STEP_NT), 0, st, k, m, ctx->hpart, ctx->hp, ctx->Hrow, colv, cS, cZ,
                       cC, ctx->gsc);
    SESM_LAUNCH_CHECK();
    slot_seq[slot] = seq;
    cplx* hout = ctx->hhost_dev + (size_t)slot * SESM_HSTRIDE;
    if (!full) {  // no update follows: publish the column on its own
      hipLaunchKernelGGL(k_gm_publish, dim3(1), dim3(256), 0, st, k + 1, colv, hout, ctx->hflag_dev + slot, seq);
      SESM_LAUNCH_CHECK();
    }
    if (full) {
      const int nrb = (N + UPD_ROWS - 1) / UPD_ROWS;
      SESM_KT_BEGIN(SESM_KT_UPDATE, st);
      hipLaunchKernelGGL(k_gm_update<VT>, dim3(nrb + (k + 1 + 3) / 4 + 1), dim3(256), 0, st, N, k, m, nrb, V, ldv,
                         cS, cZ, cC, ctx->gsc, ctx->Hrow, ctx->hp, ctx->gw, colv, hout, ctx->hflag_dev + slot, seq,
                         um);
      SESM_LAUNCH_CHECK();
      // basis V_0..V_{k-1}, u and w read; q_k and u' written
      SESM_KT_END(SESM_KT_UPDATE, st, c16 * ((double)k * N + 4.0 * N));
    }
    return SESM_OK;
  };
  auto wait_slot = [&](int slot) -> int { return gm_wait(ctx, ctx->hflag + slot, slot_seq[slot]); };
  auto take_slot = [&](int slot, int n, std::complex<double>* dst) -> int {
    return gm_take(ctx, ctx->hhost + (size_t)slot * SESM_HSTRIDE, n, dst);
  };
  using C = std::complex<double>;
  auto mul = gm_mul;
  auto rotate = gm_rotate;
  // streamed columns: raw (for the check against the device) and rotated
  // (the running residual estimate that decides when a cycle stops)
  std::vector<C>& H = ctx->gm_rot;
  std::vector<C>& Hraw = ctx->gm_raw;
  std::vector<cplx>& tri = ctx->gm_tri;
  std::vector<C> cs(m), sn(m), g(m + 1);
  auto reserve_col = [&](int j) {  // room for columns 0..j (grown geometrically, filled on use)
    const size_t need = (size_t)m_tri(j + 1);
    if (H.size() < need) H.resize(std::max(need, 2 * H.size()));
    if (Hraw.size() < need) Hraw.resize(std::max(need, 2 * Hraw.size()));
  };
  int total = 0, mismatches = 0, extra = 0;
  double est = 1.0, res_true = 1.0;
  // stopping level of the estimate in the current cycle: tol, and a quarter
  // of it in a cycle restarted from the true residual (so that a restart
  // gains more than the gap between the two residuals)
  double cyc_tol = prev_true < INFINITY ? 0.25 * tol : tol;
  bool x_zero = !warm;     // x is known to be zero (no forward map needed for its residual)
  bool r_in_v0 = false;    // V_0 already holds b - A x
  for (;;) {
    // u_0 = r = b - A x
    if (!r_in_v0) {
      if (x_zero) {
        SESM_HIP(hipMemcpyAsync(rb, b, sizeof(cplx) * (size_t)N, hipMemcpyDeviceToDevice, st));
      } else if ((rc = gm_residual(ctx, b, x, rb, inc, mixed))) {
        return rc;
      }
    }
    if (f32) {  // the stored first vector and its FP64 mirror
      hipLaunchKernelGGL(k_basis0<VT>, dim3(nb), dim3(256), 0, st, N, rb, V, um);
      SESM_LAUNCH_CHECK();
    }
    r_in_v0 = false;
    std::fill(g.begin(), g.end(), 0.0);
    {  // no step is in flight here: clear every ring slot (the last cycle's look-ahead step filled one)
      double* hv = reinterpret_cast<double*>(ctx->hhost);
      for (size_t t = 0; t < (size_t)2 * SESM_HRING * SESM_HSTRIDE; ++t) hv[t] = column_sentinel();
    }
    const int steps = std::min(m, max_iter - total);  // columns available in this cycle (0: the norm only)
    if ((rc = arnoldi(0, steps))) return rc;
    int nv = 0;
    double beta0 = 0.0, rlast = 1.0;
    for (int k = 0;; ++k) {
      if (k + 1 <= steps && (rc = arnoldi(k + 1, steps))) return rc;  // keep the device one step ahead
      const int slot = k % SESM_HRING;
      if ((rc = wait_slot(slot))) return rc;
      if (k == 0) {  // residual norm of this cycle: the true residual of x
        std::complex<double> r0;
        if ((rc = take_slot(slot, 1, &r0))) return rc;
        beta0 = r0.real();
        g[0] = beta0;
        res_true = est = beta0 / bnorm;
        if (est <= cyc_tol || steps == 0) break;
        continue;
      }
      const int j = k - 1;  // column j is final
      reserve_col(j);
      C* col = &H[(size_t)m_tri(j)];
      C* raw = &Hraw[(size_t)m_tri(j)];
      if ((rc = take_slot(slot, k + 1, raw))) return rc;
      for (int t = 0; t <= k; ++t) col[t] = raw[t];
      rlast = rotate(col, j, cs, sn, g);
      est = std::abs(g[j + 1]) / bnorm;
      nv = k;
      if (est <= cyc_tol || rlast == 0.0 || k == steps) break;
    }
    if (nv == 0) {  // x unchanged: its true residual is the cycle's initial norm
      SESM_HIP(hipStreamSynchronize(st));
      break;
    }
    // The least-squares problem is solved from the device's own Hessenberg
    // matrix (gathered after the cycle), so the update of x does not depend
    // on the streamed copies: when every streamed column equals the device's
    // bit for bit the rotations already applied stand, otherwise the
    // differing columns are counted and the rotations are redone from the
    // device's columns.  A step enqueued ahead of the last one used only
    // wrote basis vectors beyond q_{nv-1}, the step buffers and a ring slot.
    if (tri.size() < (size_t)m_tri(nv)) tri.resize((size_t)m_tri(nv));
    hipLaunchKernelGGL(k_hess_gather, dim3(nv), dim3(256), 0, st, m, ctx->Hrow, ctx->htri);
    SESM_LAUNCH_CHECK();
    SESM_HIP(hipMemcpyAsync(tri.data(), ctx->htri, sizeof(cplx) * (size_t)m_tri(nv), hipMemcpyDeviceToHost, st));
    SESM_HIP(hipStreamSynchronize(st));
    int bad = 0;
    for (int j = 0; j < nv; ++j) {
      const cplx* dv = &tri[(size_t)m_tri(j)];
      const C* raw = &Hraw[(size_t)m_tri(j)];
      bool same = true;
      for (int t = 0; t <= j + 1; ++t) same = same && C(dv[t].re, dv[t].im) == raw[t];
      bad += same ? 0 : 1;
    }
    if (bad) {
      mismatches += bad;
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta0;
      for (int j = 0; j < nv; ++j) {
        C* col = &H[(size_t)m_tri(j)];
        const cplx* dv = &tri[(size_t)m_tri(j)];
        for (int t = 0; t <= j + 1; ++t) col[t] = C(dv[t].re, dv[t].im);
        est = rotate(col, j, cs, sn, g) / bnorm;
      }
    }
    // y = R^{-1} g, x += Q y
    std::vector<C> y(nv);
    for (int t = nv - 1; t >= 0; --t) {
      C sm = g[t];
      for (int u = t + 1; u < nv; ++u) sm -= mul(H[(size_t)m_tri(u) + t], y[u]);
      y[t] = sm / H[(size_t)m_tri(t) + t];
    }
    cplx* yh = hup;  // idle: each cycle ends synchronised
    for (int t = 0; t < nv; ++t) yh[t] = cplx{y[t].real(), y[t].imag()};
    SESM_HIP(hipMemcpyAsync(ctx->ybuf, yh, sizeof(cplx) * nv, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_combine<VT>, dim3(nb), dim3(256), sizeof(cplx) * nv, st, N, nv, V, ldv, ctx->ybuf, x);
    SESM_LAUNCH_CHECK();
    total += nv;
    x_zero = false;
    // the residual of the new x (the next cycle's u_0)
    if ((rc = gm_residual(ctx, b, x, rb, inc, mixed))) return rc;
    r_in_v0 = true;
    if (est <= cyc_tol || total >= max_iter) {  // the estimate is met (or no iteration is left): check the true residual
      if ((rc = gm_rel_norm(ctx, rb, bnorm, &res_true))) return rc;
      if (res_true <= tol || total >= max_iter) break;
      // The estimate was optimistic.  A restart from the true residual helps
      // when the Krylov recurrence drifted (lost orthogonality, a clamped
      // subdiagonal); when the true residual sits at the level set by the
      // forward map's own rounding, a restart no longer lowers it.
      if (!(res_true < 0.5 * prev_true)) break;
      prev_true = res_true;
      cyc_tol = 0.25 * tol;
      ++extra;
    }
  }
  inf.iters = total;
  inf.rel_residual = res_true;
  inf.est_residual = est;
  inf.residual_restarts = extra;
  inf.column_mismatches = mismatches;
  inf.converged = res_true <= tol ? 1 : 0;
  if (info) *info = inf;
  if (!inf.converged) return ctx->fail(SESM_ENOCONV, "GMRES did not reach the tolerance");
  return SESM_OK;
}

static int solve_impl(sesm_ctx* ctx, const sesm_c64* b_in, sesm_c64* mu_out, double tol, int32_t max_iter,
                      int32_t restart, int32_t flags, double prev_true, sesm_solve_info* info, int inc = -1) {
  return solve_impl_t<cplx>(ctx, b_in, mu_out, tol, max_iter, restart, flags, prev_true, info, inc, false);
}

// Mixed precision (SESM_SOLVE_MIXED): FP64 iterative refinement around inner
// GMRES solves with an FP32 Krylov basis and the mixed-precision forward map
// (EqSources operators in FP32): r = b - A x with the FP64 map; the inner solve
// reduces ||A_mixed d - r|| by the factor tau = max(tol ||b|| / (2 ||r||), 1e-4)
// (a reduction an FP32 basis reaches reliably); x += d; repeated while the FP64
// residual at least halves.
constexpr double kMixedInnerFloor = 1e-4;
static int solve_mixed(sesm_ctx* ctx, const sesm_c64* b_in, sesm_c64* mu_out, double tol, int32_t max_iter,
                       int32_t restart, int32_t flags, sesm_solve_info* info, int inc) {
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "mixed precision needs the accelerated mode");
  if (!mu_out || !(tol > 0) || max_iter < 1 || max_iter > 100000 || restart < 0)
    return ctx->fail(SESM_EINVAL, "bad solve arguments");
  SESM_HIP(hipSetDevice(ctx->device));
  const int N = ctx->P.N;
  const int m = (restart == 0 || restart > max_iter) ? max_iter : restart;
  if (m > 4000) return ctx->fail(SESM_EINVAL, "Krylov dimension above 4000; use restart");
  int rc = ensure_workspace(ctx, m);
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  const int nb = (N + 255) / 256;
  cplx* x = (cplx*)mu_out;
  const cplx* b = (const cplx*)b_in;
  if (!b) {
    if ((rc = inc < 0 ? sesm_rhs(ctx, (sesm_c64*)ctx->wtmp) : sesm_rhs_incidence(ctx, inc, (sesm_c64*)ctx->wtmp)))
      return rc;
    b = ctx->wtmp;
  }
  double bnorm = 0.0;
  if ((rc = gm_rel_norm(ctx, b, 0.0, &bnorm))) return rc;
  if (!(flags & SESM_SOLVE_X0) || bnorm == 0.0) SESM_HIP(hipMemsetAsync(x, 0, sizeof(cplx) * (size_t)N, st));
  sesm_solve_info inf{};
  if (bnorm == 0.0) {
    SESM_HIP(hipStreamSynchronize(st));
    inf.converged = 1;
    if (info) *info = inf;
    return SESM_OK;
  }
  cplx* R = ctx->mx_R;
  cplx* D = ctx->mx_D;
  double rel = 1.0;
  if ((rc = gm_residual(ctx, b, x, R, inc, false)) || (rc = gm_rel_norm(ctx, R, bnorm, &rel))) return rc;
  int total = 0, outer = 0, mism = 0;
  double est = rel;
  while (rel > tol && total < max_iter) {
    const double tau = std::max(0.5 * tol / rel, kMixedInnerFloor);
    sesm_solve_info in{};
    rc = solve_impl_t<cplxf>(ctx, (const sesm_c64*)R, (sesm_c64*)D, tau, max_iter - total, restart, 0, INFINITY, &in,
                             inc, true);
    if (rc && rc != SESM_ENOCONV) return rc;
    total += in.iters;
    mism += in.column_mismatches;
    ++outer;
    est = in.est_residual * rel;
    hipLaunchKernelGGL(k_axpy1, dim3(nb), dim3(256), 0, st, N, x, D);
    SESM_LAUNCH_CHECK();
    double rel_new = 1.0;
    if ((rc = gm_residual(ctx, b, x, R, inc, false)) || (rc = gm_rel_norm(ctx, R, bnorm, &rel_new))) return rc;
    const bool progress = rel_new < 0.5 * rel;
    rel = rel_new;
    if (!progress || in.iters == 0) break;
  }
  inf.iters = total;
  inf.rel_residual = rel;
  inf.est_residual = est;
  inf.residual_restarts = outer;
  inf.column_mismatches = mism;
  inf.converged = rel <= tol ? 1 : 0;
  if (info) *info = inf;
  if (!inf.converged) return ctx->fail(SESM_ENOCONV, "mixed-precision GMRES did not reach the tolerance");
  return SESM_OK;
}

extern "C" int sesm_solve(sesm_ctx* ctx, const sesm_c64* b_in, sesm_c64* mu_out, double tol, int32_t max_iter,
                          int32_t restart, int32_t flags, sesm_solve_info* info) {
  if (!ctx) return SESM_EINVAL;
  if (flags & SESM_SOLVE_ADJOINT) {  // the conjugate-transpose system (dense mode)
    if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
    if (ctx->P.mode != SESM_MODE_DENSE || (flags & SESM_SOLVE_MIXED))
      return ctx->fail(SESM_EINVAL, "adjoint solves need the dense mode (and no mixed precision)");
    if (!b_in) return ctx->fail(SESM_EINVAL, "adjoint solves need a right-hand side");
    ctx->adjoint = true;
    const int rc = solve_impl(ctx, b_in, mu_out, tol, max_iter, restart, flags & ~SESM_SOLVE_ADJOINT, INFINITY, info);
    ctx->adjoint = false;
    return rc;
  }
  if (flags & SESM_SOLVE_MIXED)
    return solve_mixed(ctx, b_in, mu_out, tol, max_iter, restart, flags & ~SESM_SOLVE_MIXED, info, -1);
  return solve_impl(ctx, b_in, mu_out, tol, max_iter, restart, flags, INFINITY, info);
}

namespace {

// give a block allocated with sesm_alloc back to the context's pool
void gm_release(sesm_ctx* ctx, void* p) {
  for (size_t t = 0; t < ctx->owned.size(); ++t)
    if (ctx->owned[t].first == p) {
      ctx->bytes -= (int64_t)ctx->owned[t].second;
      sesm_pool_put(ctx, p, ctx->owned[t].second);
      ctx->owned.erase(ctx->owned.begin() + t);
      return;
    }
}

// One system of a batched solve: its device buffers (inside the batch's
// shared allocations) and its host-side state.
struct GmMember {
  void* V;          // basis (m + 1) x N, stored as the solve's VT
  cplx *w, *x;      // A u, solution
  const cplx* b;
  cplx *hcol, *hpart, *ybuf, *Hrow, *htri;  // (the step kernels derive the rest from GmBatch)
  cplx* hhost;  // pinned ring slots (+ one upload slot) and their flags
  int64_t* hflag;
  int64_t slot_seq[SESM_HRING] = {};
  std::vector<Cd> H, Hraw, cs, sn, g;
  double bnorm = 0.0, beta0 = 0.0, res = 1.0;  // res: the least-squares estimate
  double res_true = 1.0;                       // true relative residual of the final x
  int nv = 0, mism = 0;
  bool active = false;
};

}  // namespace

// inc0 >= 0: system r uses the operator of member inc0 + r of the incidence
// set (b may then be NULL: each member's incident field).  VT: storage of the
// bases (cplxf: the inner solves of mixed precision, whose forward maps are
// the mixed-precision ones when mixed is set and read the FP64 mirrors Umir).
template <typename VT>
static int solve_batch_impl(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* b_in, int64_t ld_b, sesm_c64* mu_out,
                            int64_t ld_mu, double tol, int32_t max_iter, int32_t flags, sesm_solve_info* info,
                            int inc0, bool mixed = false) {
  constexpr bool f32 = !std::is_same<VT, cplx>::value;
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (nrhs < 0 || nrhs > SESM_MAX_BATCH || !(tol > 0) || max_iter < 1 || max_iter > 4000 ||
      (flags & ~SESM_SOLVE_X0))
    return ctx->fail(SESM_EINVAL, "bad batched solve arguments");
  const bool warm = (flags & SESM_SOLVE_X0) != 0;
  if (nrhs == 0) return SESM_OK;
  const int N = ctx->P.N;
  if ((!b_in && inc0 < 0) || !mu_out || ld_b < N || ld_mu < N)
    return ctx->fail(SESM_EINVAL, "bad batched solve arguments");
  if (b_in) {  // the spans of the right-hand sides and of the solutions must be disjoint
    const uintptr_t b0 = (uintptr_t)b_in, b1 = (uintptr_t)(b_in + (nrhs - 1) * ld_b + N);
    const uintptr_t m0 = (uintptr_t)mu_out, m1 = (uintptr_t)(mu_out + (nrhs - 1) * ld_mu + N);
    if (b0 < m1 && m0 < b1) return ctx->fail(SESM_EINVAL, "right-hand sides and solutions overlap");
  }
  SESM_HIP(hipSetDevice(ctx->device));
  const int m = max_iter;
  hipStream_t st = ctx->stream;
  const int nb = (N + 255) / 256;
  const int64_t ldv = N, vstride = (int64_t)(m + 1) * N;
  // per-member small buffers, each rounded to 16 complex entries
  auto r16 = [](int64_t n) { return (n + 15) / 16 * 16; };
  const int64_t hrow_len = hrow_off(m, m) + 1;
  const int64_t o_hcol = 0, o_hpart = o_hcol + r16((int64_t)SESM_HRING * SESM_HSTRIDE),
                o_ybuf = o_hpart + r16((int64_t)2 * SESM_HSTRIDE * DCHUNK), o_hp = o_ybuf + r16(SESM_HSTRIDE),
                o_gcoef = o_hp + r16(SESM_HSTRIDE), o_gsc = o_gcoef + r16(3 * SESM_HSTRIDE), o_Hrow = o_gsc + 16,
                o_htri = o_Hrow + r16(hrow_len), per_small = o_htri + r16(m_tri(m));
  VT* Vall = nullptr;
  cplx *Wall = nullptr, *small = nullptr, *Umir = nullptr;
  cplx* pin = nullptr;
  int rc = SESM_OK;
  std::vector<GmMember> M(nrhs);
  auto finish = [&](int code) -> int {  // free the workspace (after the stream has drained)
    (void)hipStreamSynchronize(st);
    if (pin) (void)hipHostFree(pin);
    gm_release(ctx, Vall);
    gm_release(ctx, Wall);
    gm_release(ctx, small);
    gm_release(ctx, Umir);
    return code;
  };
  // the members' incident fields when no right-hand sides are given (kept
  // until a system continuing alone has finished)
  cplx* Ball = nullptr;
  auto finish_all = [&](int code) -> int {
    const int c = finish(code);
    gm_release(ctx, Ball);
    return c;
  };
  if (!b_in) {
    if ((rc = sesm_alloc(ctx, (void**)&Ball, sizeof(cplx) * (size_t)nrhs * N))) return rc;
    for (int r = 0; r < nrhs; ++r)
      if ((rc = sesm_rhs_incidence(ctx, inc0 + r, (sesm_c64*)(Ball + (int64_t)r * N)))) return finish_all(rc);
    b_in = (const sesm_c64*)Ball;
    ld_b = N;
  }
  if ((rc = sesm_alloc(ctx, (void**)&Vall, sizeof(VT) * (size_t)nrhs * vstride)) ||
      (rc = sesm_alloc(ctx, (void**)&Wall, sizeof(cplx) * (size_t)nrhs * N)) ||
      (rc = sesm_alloc(ctx, (void**)&small, sizeof(cplx) * (size_t)nrhs * per_small)) ||
      (f32 && (rc = sesm_alloc(ctx, (void**)&Umir, sizeof(cplx) * (size_t)nrhs * N))))
    return finish_all(rc);
  const size_t pin_per = (size_t)(SESM_HRING + 1) * SESM_HSTRIDE + SESM_HRING;  // slots, then flags (as cplx)
  if (hipHostMalloc((void**)&pin, sizeof(cplx) * pin_per * nrhs, hipHostMallocCoherent) != hipSuccess) {
    pin = nullptr;
    return finish_all(ctx->fail(SESM_ENOMEM, "hipHostMalloc failed"));
  }
  cplx* pin_dev = nullptr;
  if (hipHostGetDevicePointer((void**)&pin_dev, pin, 0) != hipSuccess)
    return finish_all(ctx->fail(SESM_EHIP, "hipHostGetDevicePointer failed"));
  for (int r = 0; r < nrhs; ++r) {
    GmMember& G = M[r];
    G.V = Vall + r * vstride;
    G.w = Wall + (int64_t)r * N;
    G.x = (cplx*)mu_out + r * ld_mu;
    G.b = (const cplx*)b_in + r * ld_b;
    cplx* sm = small + r * per_small;
    G.hcol = sm + o_hcol;
    G.hpart = sm + o_hpart;
    G.ybuf = sm + o_ybuf;
    G.Hrow = sm + o_Hrow;
    G.htri = sm + o_htri;
    G.hhost = pin + r * pin_per;
    G.hflag = reinterpret_cast<int64_t*>(G.hhost + (size_t)(SESM_HRING + 1) * SESM_HSTRIDE);
    for (int t = 0; t < SESM_HRING; ++t) G.hflag[t] = 0;
    double* hv = reinterpret_cast<double*>(G.hhost);
    for (size_t t = 0; t < (size_t)2 * SESM_HRING * SESM_HSTRIDE; ++t) hv[t] = column_sentinel();
    G.cs.assign(m, 0.0);
    G.sn.assign(m, 0.0);
    G.g.assign(m + 1, 0.0);
    // right-hand side norm and u_0 = b (x = 0)
    hipLaunchKernelGGL(k_norm2_part, dim3(NCHUNK), dim3(256), 0, st, N, G.b, (double*)G.hpart);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, (const double*)G.hpart, G.hcol);
    if (hipGetLastError() != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: launch failed"));
    cplx* hup = G.hhost + (size_t)SESM_HRING * SESM_HSTRIDE;
    if (hipMemcpyAsync(hup, G.hcol, sizeof(cplx), hipMemcpyDeviceToHost, st) != hipSuccess)
      return finish_all(ctx->fail(SESM_EHIP, "batched solve: initial copies failed"));
  }
  if (hipStreamSynchronize(st) != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: synchronisation failed"));
  for (int r = 0; r < nrhs; ++r) {
    M[r].bnorm = M[r].hhost[(size_t)SESM_HRING * SESM_HSTRIDE].re;
    M[r].active = M[r].bnorm != 0.0;
    M[r].res = M[r].bnorm != 0.0 ? 1.0 : 0.0;
  }
  // u_0 = b - A x for every system: b itself from x = 0, or (warm start) one
  // batched forward map of the initial guesses; a zero right-hand side has
  // the solution 0
  if (warm) {
    int r2 = SESM_OK;
    if (ctx->P.mode == SESM_MODE_ACCEL)
      r2 = sesm_accel_matvec_batch(ctx, nrhs, (const cplx*)mu_out, ld_mu, Wall, N, inc0, mixed);
    else
      for (int r = 0; r < nrhs && !r2; ++r) r2 = sesm_dense_matvec(ctx, M[r].x, M[r].w);
    if (r2) return finish_all(r2);
  }
  for (int r = 0; r < nrhs; ++r) {
    GmMember& G = M[r];
    cplx* um = f32 ? Umir + (int64_t)r * N : nullptr;
    if (warm && G.bnorm != 0.0) {
      hipLaunchKernelGGL(k_sub_from, dim3(nb), dim3(256), 0, st, N, G.b, G.w);
      hipLaunchKernelGGL(k_basis0<VT>, dim3(nb), dim3(256), 0, st, N, G.w, (VT*)G.V, um);
      if (hipGetLastError() != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: initial residual failed"));
    } else {
      hipLaunchKernelGGL(k_basis0<VT>, dim3(nb), dim3(256), 0, st, N, G.b, (VT*)G.V, um);
      if (hipGetLastError() != hipSuccess || hipMemsetAsync(G.x, 0, sizeof(cplx) * (size_t)N, st) != hipSuccess)
        return finish_all(ctx->fail(SESM_EHIP, "batched solve: initial copies failed"));
    }
  }
  GmBatch GB0{};
  GB0.V = Vall;
  GB0.U = Umir;
  GB0.vstride = vstride;
  GB0.W = Wall;
  GB0.small = small;
  GB0.sstride = per_small;
  GB0.o_hcol = o_hcol;
  GB0.o_hpart = o_hpart;
  GB0.o_hp = o_hp;
  GB0.o_gcoef = o_gcoef;
  GB0.o_gsc = o_gsc;
  GB0.o_Hrow = o_Hrow;
  GB0.pin = pin_dev;
  GB0.pstride = (int64_t)pin_per;
  const int steps = m;  // unrestarted: every column of the basis is available
  // Arnoldi step k of every active member: one batched forward map of the
  // members' u = V_k, then each member's dot products, step and update (the
  // same launches as the single solve, on the member's buffers).
  auto arnoldi_all = [&](int k) -> int {
    const bool full = k < steps;
    int lo = nrhs, hi = -1;
    for (int r = 0; r < nrhs; ++r)
      if (M[r].active) lo = std::min(lo, r), hi = std::max(hi, r);
    if (hi < 0) return SESM_OK;
    if (full) {
      int r2;
      if (ctx->P.mode == SESM_MODE_ACCEL)
        r2 = f32 ? sesm_accel_matvec_batch(ctx, hi - lo + 1, Umir + (int64_t)lo * N, N, Wall + (int64_t)lo * N, N,
                                           inc0 < 0 ? -1 : inc0 + lo, mixed)
                 : sesm_accel_matvec_batch(ctx, hi - lo + 1, (const cplx*)(Vall + lo * vstride + (int64_t)k * ldv),
                                           vstride, Wall + (int64_t)lo * N, N, inc0 < 0 ? -1 : inc0 + lo, mixed);
      else {
        r2 = SESM_OK;
        for (int r = lo; r <= hi && !r2; ++r)
          r2 = sesm_dense_matvec(ctx, (const cplx*)M[r].V + (int64_t)k * ldv, M[r].w);  // (FP64 bases only)
      }
      if (r2) return r2;
    }
    // the members' dot products, steps and updates: one launch each for all
    // active members (member i of the mask gets sequence number seq0 + i)
    const int slot = k % SESM_HRING;
    GmBatch GB = GB0;
    GB.seq0 = ctx->gm_seq + 1;
    GB.active = 0;
    int na = 0;
    for (int r = 0; r < nrhs; ++r)
      if (M[r].active) {
        GB.active |= 1ull << r;
        M[r].slot_seq[slot] = GB.seq0 + na++;
      }
    ctx->gm_seq += na;
    hipLaunchKernelGGL(k_gm_dots_batch<VT>, dim3(DCHUNK, (k + 1 + VB - 1) / VB, na), dim3(256), 0, st, GB, N, k,
                       full ? 1 : 0);
    SESM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gm_step_batch, dim3(na), dim3(STEP_NT), 0, st, GB, k, m);
    SESM_LAUNCH_CHECK();
    if (!full) {
      hipLaunchKernelGGL(k_gm_publish_batch, dim3(na), dim3(256), 0, st, GB, k);
    } else {
      const int nrb = (N + UPD_ROWS - 1) / UPD_ROWS;
      hipLaunchKernelGGL(k_gm_update_batch<VT>, dim3(nrb + (k + 1 + 3) / 4 + 1, 1, na), dim3(256), 0, st, GB, N, k, m,
                         nrb);
    }
    SESM_LAUNCH_CHECK();
    return SESM_OK;
  };
  if ((rc = arnoldi_all(0))) return finish_all(rc);
  int active = 0;
  for (const GmMember& G : M) active += G.active ? 1 : 0;
  for (int k = 0; active > 0; ++k) {
    if (k + 1 <= steps && (rc = arnoldi_all(k + 1))) return finish_all(rc);  // the device stays one step ahead
    const int slot = k % SESM_HRING;
    for (int r = 0; r < nrhs; ++r) {
      GmMember& G = M[r];
      if (!G.active) continue;
      if ((rc = gm_wait(ctx, G.hflag + slot, G.slot_seq[slot]))) return finish_all(rc);
      cplx* hs = G.hhost + (size_t)slot * SESM_HSTRIDE;
      if (k == 0) {  // residual norm
        Cd r0;
        if ((rc = gm_take(ctx, hs, 1, &r0))) return finish_all(rc);
        G.beta0 = r0.real();
        G.g[0] = G.beta0;
        G.res = G.res_true = G.beta0 / G.bnorm;
        if (G.res <= tol) G.active = false, --active;
        continue;
      }
      const int j = k - 1;
      const size_t need = (size_t)m_tri(j + 1);
      if (G.H.size() < need) G.H.resize(std::max(need, 2 * G.H.size()));
      if (G.Hraw.size() < need) G.Hraw.resize(std::max(need, 2 * G.Hraw.size()));
      Cd* col = &G.H[(size_t)m_tri(j)];
      Cd* raw = &G.Hraw[(size_t)m_tri(j)];
      if ((rc = gm_take(ctx, hs, k + 1, raw))) return finish_all(rc);
      for (int t = 0; t <= k; ++t) col[t] = raw[t];
      const double rr = gm_rotate(col, j, G.cs, G.sn, G.g);
      G.res = std::abs(G.g[j + 1]) / G.bnorm;
      G.nv = k;
      if (G.res <= tol || rr == 0.0 || k == steps) G.active = false, --active;
    }
  }
  // per member: least squares from the device's own Hessenberg columns
  // (streamed copies compared bitwise), x = V y
  std::vector<cplx> tri;
  for (int r = 0; r < nrhs; ++r) {
    GmMember& G = M[r];
    const int nv = G.nv;
    if (nv == 0) continue;
    if (tri.size() < (size_t)m_tri(nv)) tri.resize((size_t)m_tri(nv));
    hipLaunchKernelGGL(k_hess_gather, dim3(nv), dim3(256), 0, st, m, G.Hrow, G.htri);
    if (hipGetLastError() != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: launch failed"));
    if (hipMemcpyAsync(tri.data(), G.htri, sizeof(cplx) * (size_t)m_tri(nv), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return finish_all(ctx->fail(SESM_EHIP, "batched solve: Hessenberg transfer failed"));
    int bad = 0;
    for (int j = 0; j < nv; ++j) {
      const cplx* dv = &tri[(size_t)m_tri(j)];
      const Cd* raw = &G.Hraw[(size_t)m_tri(j)];
      bool same = true;
      for (int t = 0; t <= j + 1; ++t) same = same && Cd(dv[t].re, dv[t].im) == raw[t];
      bad += same ? 0 : 1;
    }
    if (bad) {
      G.mism += bad;
      std::fill(G.g.begin(), G.g.end(), 0.0);
      G.g[0] = G.beta0;
      for (int j = 0; j < nv; ++j) {
        Cd* col = &G.H[(size_t)m_tri(j)];
        const cplx* dv = &tri[(size_t)m_tri(j)];
        for (int t = 0; t <= j + 1; ++t) col[t] = Cd(dv[t].re, dv[t].im);
        G.res = gm_rotate(col, j, G.cs, G.sn, G.g) / G.bnorm;
      }
    }
    std::vector<Cd> y(nv);
    for (int t = nv - 1; t >= 0; --t) {
      Cd sm = G.g[t];
      for (int u = t + 1; u < nv; ++u) sm -= gm_mul(G.H[(size_t)m_tri(u) + t], y[u]);
      y[t] = sm / G.H[(size_t)m_tri(t) + t];
    }
    cplx* yh = G.hhost + (size_t)SESM_HRING * SESM_HSTRIDE;
    for (int t = 0; t < nv; ++t) yh[t] = cplx{y[t].real(), y[t].imag()};
    if (hipMemcpyAsync(G.ybuf, yh, sizeof(cplx) * nv, hipMemcpyHostToDevice, st) != hipSuccess)
      return finish_all(ctx->fail(SESM_EHIP, "batched solve: upload failed"));
    hipLaunchKernelGGL(k_combine<VT>, dim3(nb), dim3(256), sizeof(cplx) * nv, st, N, nv, (const VT*)G.V, ldv, G.ybuf,
                       G.x);
    if (hipGetLastError() != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: launch failed"));
    if (hipStreamSynchronize(st) != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: combine failed"));
  }
  // true residuals b - A x of the updated systems: one batched forward map of
  // all solutions, then each updated system's norm (the others' true residual
  // is their initial norm)
  {
    int r2 = SESM_OK;
    if (ctx->P.mode == SESM_MODE_ACCEL)
      r2 = sesm_accel_matvec_batch(ctx, nrhs, (const cplx*)mu_out, ld_mu, Wall, N, inc0, mixed);
    else
      for (int r = 0; r < nrhs && !r2; ++r)
        if (M[r].nv > 0) r2 = sesm_dense_matvec(ctx, M[r].x, M[r].w);
    if (r2) return finish_all(r2);
    for (int r = 0; r < nrhs; ++r) {
      GmMember& G = M[r];
      if (G.nv == 0) continue;
      hipLaunchKernelGGL(k_sub_from, dim3(nb), dim3(256), 0, st, N, G.b, G.w);
      hipLaunchKernelGGL(k_norm2_part, dim3(NCHUNK), dim3(256), 0, st, N, G.w, (double*)G.hpart);
      hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, (const double*)G.hpart, G.hcol);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(G.hhost + (size_t)SESM_HRING * SESM_HSTRIDE, G.hcol, sizeof(cplx), hipMemcpyDeviceToHost,
                         st) != hipSuccess)
        return finish_all(ctx->fail(SESM_EHIP, "batched solve: residual check failed"));
    }
    if (hipStreamSynchronize(st) != hipSuccess) return finish_all(ctx->fail(SESM_EHIP, "batched solve: residual check failed"));
    for (int r = 0; r < nrhs; ++r)
      if (M[r].nv > 0) M[r].res_true = M[r].hhost[(size_t)SESM_HRING * SESM_HSTRIDE].re / M[r].bnorm;
  }
  rc = finish(SESM_OK);
  if (rc) return rc;
  // a system whose estimate was met but whose true residual is not continues
  // alone from its solution with restarted cycles (as sesm_solve would)
  bool all = true;
  for (int r = 0; r < nrhs; ++r) {
    GmMember& G = M[r];
    sesm_solve_info more{};
    int extra = 0, iters = G.nv, mism = G.mism;
    double res_true = G.res_true, est = G.res;
    if (G.bnorm != 0.0 && res_true > tol && G.nv > 0 && G.nv < max_iter) {
      const int r2 = solve_impl_t<VT>(ctx, (const sesm_c64*)G.b, (sesm_c64*)G.x, tol, max_iter - G.nv, 0, SESM_SOLVE_X0,
                                      G.res_true, &more, inc0 < 0 ? -1 : inc0 + r, mixed);
      if (r2 && r2 != SESM_ENOCONV) {
        gm_release(ctx, Ball);
        return r2;
      }
      extra = 1 + more.residual_restarts;
      iters += more.iters;
      mism += more.column_mismatches;
      res_true = more.rel_residual;
      est = more.est_residual;
    }
    if (G.bnorm == 0.0) res_true = est = 0.0;
    const bool conv = res_true <= tol;
    all = all && conv;
    if (info) {
      info[r] = sesm_solve_info{};
      info[r].iters = iters;
      info[r].rel_residual = res_true;
      info[r].est_residual = est;
      info[r].residual_restarts = extra;
      info[r].converged = conv ? 1 : 0;
      info[r].column_mismatches = mism;
    }
  }
  gm_release(ctx, Ball);
  if (!all) return ctx->fail(SESM_ENOCONV, "GMRES did not reach the tolerance for every right-hand side");
  return SESM_OK;
}

// Mixed precision for a batch: FP64 refinement around lockstep inner solves
// with FP32 bases and the mixed-precision map (as solve_mixed, one
// refinement step for all systems that have not yet reached tol; a system
// stops when its FP64 residual fails to halve).
static int solve_batch_mixed(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* b_in, int64_t ld_b, sesm_c64* mu_out,
                             int64_t ld_mu, double tol, int32_t max_iter, int32_t flags, sesm_solve_info* info,
                             int inc0) {
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "mixed precision needs the accelerated mode");
  if (nrhs < 0 || nrhs > SESM_MAX_BATCH || !(tol > 0) || max_iter < 1 || max_iter > 4000)
    return ctx->fail(SESM_EINVAL, "bad batched solve arguments");
  if (nrhs == 0) return SESM_OK;
  const int N = ctx->P.N;
  if ((!b_in && inc0 < 0) || !mu_out || ld_mu < N || (b_in && ld_b < N))
    return ctx->fail(SESM_EINVAL, "bad batched solve arguments");
  SESM_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int nb = (N + 255) / 256;
  int rc = ensure_small(ctx);  // (norms go through the small buffers)
  if (rc) return rc;
  cplx *B = nullptr, *R = nullptr, *D = nullptr;
  auto done = [&](int code) -> int {
    (void)hipStreamSynchronize(st);
    gm_release(ctx, B);
    gm_release(ctx, R);
    gm_release(ctx, D);
    return code;
  };
  if ((rc = sesm_alloc(ctx, (void**)&B, sizeof(cplx) * (size_t)nrhs * N)) ||
      (rc = sesm_alloc(ctx, (void**)&R, sizeof(cplx) * (size_t)nrhs * N)) ||
      (rc = sesm_alloc(ctx, (void**)&D, sizeof(cplx) * (size_t)nrhs * N)))
    return done(rc);
  // right-hand sides (given or the members' incident fields), initial x
  for (int r = 0; r < nrhs; ++r) {
    cplx* br = B + (int64_t)r * N;
    if (b_in) {
      SESM_HIP(hipMemcpyAsync(br, (const cplx*)b_in + r * ld_b, sizeof(cplx) * N, hipMemcpyDeviceToDevice, st));
    } else if ((rc = sesm_rhs_incidence(ctx, inc0 + r, (sesm_c64*)br))) {
      return done(rc);
    }
    if (!(flags & SESM_SOLVE_X0)) SESM_HIP(hipMemsetAsync((cplx*)mu_out + r * ld_mu, 0, sizeof(cplx) * N, st));
  }
  std::vector<double> bn(nrhs), rel(nrhs, 1.0), est(nrhs, 1.0);
  std::vector<int> iters(nrhs, 0), steps(nrhs, 0), mism(nrhs, 0);
  std::vector<char> active(nrhs, 1);
  auto residuals = [&]() -> int {  // R = B - A X with the FP64 map, and the relative norms
    int r2 = sesm_accel_matvec_batch(ctx, nrhs, (const cplx*)mu_out, ld_mu, R, N, inc0, false);
    if (r2) return r2;
    for (int r = 0; r < nrhs; ++r) {
      hipLaunchKernelGGL(k_sub_from, dim3(nb), dim3(256), 0, st, N, B + (int64_t)r * N, R + (int64_t)r * N);
      SESM_LAUNCH_CHECK();
      double v = 0.0;
      if ((r2 = gm_rel_norm(ctx, R + (int64_t)r * N, bn[r], &v))) return r2;
      if (active[r]) rel[r] = v;
    }
    return SESM_OK;
  };
  for (int r = 0; r < nrhs; ++r)
    if ((rc = gm_rel_norm(ctx, B + (int64_t)r * N, 0.0, &bn[r]))) return done(rc);
  for (int r = 0; r < nrhs; ++r) active[r] = bn[r] > 0.0;
  if ((rc = residuals())) return done(rc);
  std::vector<sesm_solve_info> in(nrhs);
  for (int used = 0;;) {
    double worst = 0.0;
    int n_act = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (active[r] && rel[r] <= tol) active[r] = 0;
      if (active[r]) worst = std::max(worst, rel[r]), ++n_act;
    }
    if (n_act == 0 || used >= max_iter) break;
    // systems that are done get a zero right-hand side (their correction is 0)
    for (int r = 0; r < nrhs; ++r)
      if (!active[r]) SESM_HIP(hipMemsetAsync(R + (int64_t)r * N, 0, sizeof(cplx) * N, st));
    const double tau = std::max(0.5 * tol / worst, kMixedInnerFloor);
    rc = solve_batch_impl<cplxf>(ctx, nrhs, (const sesm_c64*)R, N, (sesm_c64*)D, N, tau, max_iter - used, 0,
                                 in.data(), inc0, true);
    if (rc && rc != SESM_ENOCONV) return done(rc);
    int most = 0;
    std::vector<double> before(rel);
    for (int r = 0; r < nrhs; ++r) {
      if (!active[r]) continue;
      hipLaunchKernelGGL(k_axpy1, dim3(nb), dim3(256), 0, st, N, (cplx*)mu_out + r * ld_mu, D + (int64_t)r * N);
      SESM_LAUNCH_CHECK();
      iters[r] += in[r].iters;
      mism[r] += in[r].column_mismatches;
      ++steps[r];
      est[r] = in[r].est_residual * rel[r];
      most = std::max(most, in[r].iters);
    }
    used += most;
    if ((rc = residuals())) return done(rc);
    for (int r = 0; r < nrhs; ++r)
      if (active[r] && (!(rel[r] < 0.5 * before[r]) || in[r].iters == 0)) active[r] = 0;  // no progress
  }
  bool all = true;
  for (int r = 0; r < nrhs; ++r) {
    const bool conv = bn[r] == 0.0 || rel[r] <= tol;
    all = all && conv;
    if (info) {
      info[r] = sesm_solve_info{};
      info[r].iters = iters[r];
      info[r].rel_residual = bn[r] == 0.0 ? 0.0 : rel[r];
      info[r].est_residual = bn[r] == 0.0 ? 0.0 : est[r];
      info[r].residual_restarts = steps[r];
      info[r].column_mismatches = mism[r];
      info[r].converged = conv ? 1 : 0;
    }
  }
  rc = done(SESM_OK);
  if (rc) return rc;
  if (!all) return ctx->fail(SESM_ENOCONV, "mixed-precision GMRES did not reach the tolerance for every system");
  return SESM_OK;
}

extern "C" int sesm_solve_batch(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* b, int64_t ld_b, sesm_c64* mu,
                                int64_t ld_mu, double tol, int32_t max_iter, int32_t flags, sesm_solve_info* info) {
  if (!ctx) return SESM_EINVAL;
  if (flags & SESM_SOLVE_MIXED)
    return solve_batch_mixed(ctx, nrhs, b, ld_b, mu, ld_mu, tol, max_iter, flags & ~SESM_SOLVE_MIXED, info, -1);
  return solve_batch_impl<cplx>(ctx, nrhs, b, ld_b, mu, ld_mu, tol, max_iter, flags, info, -1);
}

extern "C" int sesm_solve_incidences(sesm_ctx* ctx, int32_t r0, int32_t nrhs, const sesm_c64* b, int64_t ld_b,
                                     sesm_c64* mu, int64_t ld_mu, double tol, int32_t max_iter, int32_t flags,
                                     sesm_solve_info* info) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL) return ctx->fail(SESM_EINVAL, "incidence sets need the accelerated mode");
  if (r0 < 0 || nrhs < 0 || r0 + nrhs > sesm_accel_n_incidences(ctx))
    return ctx->fail(SESM_EINVAL, "incidence index beyond the incidence set");
  if (!b) ld_b = ctx->P.N;
  if (flags & SESM_SOLVE_MIXED)
    return solve_batch_mixed(ctx, nrhs, b, ld_b, mu, ld_mu, tol, max_iter, flags & ~SESM_SOLVE_MIXED, info, r0);
  return solve_batch_impl<cplx>(ctx, nrhs, b, ld_b, mu, ld_mu, tol, max_iter, flags, info, r0);
}
