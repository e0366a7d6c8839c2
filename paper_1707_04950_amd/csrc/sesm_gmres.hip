// GMRES (Algorithm 1: "Run GMRES iterations, using the forward map").
//
// Device-resident Krylov basis V[(m+1) x N]; classical Gram-Schmidt applied
// twice (CGS2) with tall-skinny dot-product kernels (each kernel reads every
// basis vector once, coalesced); Givens rotations of the small Hessenberg
// matrix on the host, which reads one column per iteration.  The host runs one
// Arnoldi step behind the device: step it+1 is enqueued before the column of
// step it is read back, so the device never waits for the host's rotations
// (the extra step after convergence is discarded).
#include <cmath>
#include <complex>
#include <vector>

#include "sesm_impl.h"

namespace {

constexpr int VT = 8;         // basis vectors per dot-product block
constexpr int NCHUNK = 240;   // N-chunks of the single-vector norm reduction
constexpr int DCHUNK = 32;    // N-chunks of the multi-vector dot products (about 1 KB of w per block)

// part[v * DCHUNK + c] = sum_{i in chunk c} conj(V_v[i]) w[i], v in [0, nv).
// Loads are unconditional (vector index clamped, surplus terms masked) so that
// all VT basis loads of an iteration are in flight together.
__global__ __launch_bounds__(256) void k_dots(int N, int nv, const cplx* __restrict__ V, int64_t ldv,
                                              const cplx* __restrict__ w, cplx* __restrict__ part) {
  __shared__ cplx sh[VT][4];
  const int c = blockIdx.x, v0 = blockIdx.y * VT;
  const int per = (N + DCHUNK - 1) / DCHUNK;
  const int lo = c * per, hi = min(N, lo + per);
  const cplx* row[VT];
  double msk[VT];
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    row[t] = V + (int64_t)min(v0 + t, nv - 1) * ldv;
    msk[t] = v0 + t < nv ? 1.0 : 0.0;
  }
  cplx acc[VT];
#pragma unroll
  for (int t = 0; t < VT; ++t) acc[t] = cplx{0.0, 0.0};
  // two elements per thread and step: all 2 VT basis loads are issued before any use
  for (int i = lo + threadIdx.x; i < hi; i += 512) {
    const bool two = i + 256 < hi;
    const int i2 = two ? i + 256 : i;
    cplx a[VT], b[VT];
#pragma unroll
    for (int t = 0; t < VT; ++t) a[t] = row[t][i];
#pragma unroll
    for (int t = 0; t < VT; ++t) b[t] = row[t][i2];
    const cplx wa = w[i];
    const cplx wb = two ? w[i2] : cplx{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < VT; ++t) acc[t] += cmul_conj(a[t], wa) + cmul_conj(b[t], wb);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    const cplx s = wave_sum(acc[t]);
    if (lane == 0) sh[t][wv] = msk[t] * s;
  }
  __syncthreads();
  if (threadIdx.x < VT && v0 + (int)threadIdx.x < nv) {
    const int t = threadIdx.x;
    part[(int64_t)(v0 + t) * DCHUNK + c] = sh[t][0] + sh[t][1] + sh[t][2] + sh[t][3];
  }
}

// upart[c][i] = sum_{v in chunk c} V_v[i] coef[v], chunks of UCH vectors (more
// workgroups than one pass over all vectors, and independent loads in flight).
// Each workgroup first reduces the dot-product partials of its chunk,
// coef[v] = sum_c' dpart[v * DCHUNK + c'] (one wave per v); the workgroups with
// blockIdx.x == 0 also store h[v] = coef[v] (first pass) or h[v] + coef[v].
constexpr int UCH = 32;
__global__ __launch_bounds__(256) void k_update_part(int N, int nv, const cplx* __restrict__ V, int64_t ldv,
                                                     const cplx* __restrict__ dpart, cplx* __restrict__ h,
                                                     int accumulate, cplx* __restrict__ upart) {
  __shared__ cplx hs[UCH];
  const int c = blockIdx.y;
  const int v0 = c * UCH, v1 = min(nv, v0 + UCH);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int v = v0 + wv; v < v1; v += 4) {
    cplx sm = lane < DCHUNK ? dpart[(int64_t)v * DCHUNK + lane] : cplx{0.0, 0.0};
    sm = wave_sum(sm);
    if (lane == 0) {
      hs[v - v0] = sm;
      if (blockIdx.x == 0) h[v] = accumulate ? h[v] + sm : sm;
    }
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  cplx sm = cplx{0.0, 0.0};
#pragma unroll 8
  for (int v = v0; v < v1; ++v) sm += V[(int64_t)v * ldv + i] * hs[v - v0];
  upart[(int64_t)c * N + i] = sm;
}

// w[i] -= sum_c part[c][i]; with npart, also npart[block] = sum over the block of |w[i]|^2
__global__ __launch_bounds__(256) void k_update_final(int N, int nch, const cplx* __restrict__ part,
                                                      cplx* __restrict__ w, double* __restrict__ npart) {
  __shared__ cplx sh[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double q = 0.0;
  if (i < N) {
    cplx s = w[i];
    for (int c = 0; c < nch; ++c) s -= part[(int64_t)c * N + i];
    w[i] = s;
    q = abs2(s);
  }
  if (npart) {
    const cplx r = block_sum<256>(cplx{q, 0.0}, sh);
    if (threadIdx.x == 0) npart[blockIdx.x] = r.re;
  }
}

// n = sqrt(sum of the nparts partial squared norms); w /= n (zero norm leaves w);
// block 0 stores cplx(n, 0) at *hout
__global__ __launch_bounds__(256) void k_scale_norm(int N, int nparts, const double* __restrict__ npart, cplx* w,
                                                    cplx* __restrict__ hout) {
  __shared__ cplx sh[4];
  __shared__ double nrm;
  double s = 0.0;
  for (int c = threadIdx.x; c < nparts; c += 256) s += npart[c];
  const cplx r = block_sum<256>(cplx{s, 0.0}, sh);
  if (threadIdx.x == 0) {
    nrm = sqrt(r.re);
    if (blockIdx.x == 0) *hout = cplx{nrm, 0.0};
  }
  __syncthreads();
  const double n = nrm;
  const double inv = n > 0 ? 1.0 / n : 0.0;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N && n > 0) w[i] = inv * w[i];
}

// x[i] += sum_{v < nv} V_v[i] y[v]
__global__ __launch_bounds__(256) void k_combine(int N, int nv, const cplx* __restrict__ V, int64_t ldv,
                                                 const cplx* __restrict__ y, cplx* __restrict__ x, int add) {
  extern __shared__ cplx ys[];
  for (int v = threadIdx.x; v < nv; v += 256) ys[v] = y[v];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  cplx s = add ? x[i] : cplx{0.0, 0.0};
  for (int v = 0; v < nv; ++v) s += V[(int64_t)v * ldv + i] * ys[v];
  x[i] = s;
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

// dst = src / norm (norm read from device; zero norm leaves zeros)
__global__ void k_scale(int N, const cplx* src, const cplx* __restrict__ nrm, cplx* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double n = nrm->re;
  const double s = n > 0 ? 1.0 / n : 0.0;
  dst[i] = s * src[i];
}

// r = b - r
__global__ void k_sub_from(int N, const cplx* __restrict__ b, cplx* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  r[i] = b[i] - r[i];
}

int ensure_workspace(sesm_ctx* ctx, int m) {
  const int N = ctx->P.N;
  if (ctx->V && ctx->V_cols >= m + 1) return SESM_OK;
  auto drop = [&](void* p) {
    if (!p) return;
    for (size_t t = 0; t < ctx->owned.size(); ++t)
      if (ctx->owned[t] == p) {
        ctx->owned.erase(ctx->owned.begin() + t);
        break;
      }
    (void)hipFree(p);
  };
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->V) ctx->bytes -= (int64_t)ctx->V_cols * N * (int64_t)sizeof(cplx);
  drop(ctx->V);
  ctx->V = nullptr;
  ctx->V_cols = 0;
  int rc = sesm_alloc(ctx, (void**)&ctx->V, sizeof(cplx) * (size_t)(m + 1) * N);
  if (rc) return rc;
  ctx->V_cols = m + 1;
  if (!ctx->hcol) {
    if ((rc = sesm_alloc(ctx, (void**)&ctx->hcol, sizeof(cplx) * SESM_HRING * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->hpart, sizeof(cplx) * (size_t)SESM_HSTRIDE * DCHUNK))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->ybuf, sizeof(cplx) * SESM_HSTRIDE))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->wtmp, sizeof(cplx) * (size_t)N))) return rc;
    if ((rc = sesm_alloc(ctx, (void**)&ctx->upart, sizeof(cplx) * (size_t)N * ((SESM_HSTRIDE + UCH - 1) / UCH))))
      return rc;
    if (hipHostMalloc((void**)&ctx->hhost, sizeof(cplx) * (SESM_HRING + 1) * SESM_HSTRIDE, 0) != hipSuccess)
      return ctx->fail(SESM_ENOMEM, "hipHostMalloc failed");
    for (hipEvent_t& ev : ctx->hev)
      if (!ev) SESM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  return SESM_OK;
}

}  // namespace

extern "C" int sesm_solve(sesm_ctx* ctx, const sesm_c64* b_in, sesm_c64* mu_out, double tol, int32_t max_iter,
                          int32_t restart, sesm_solve_info* info) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (!mu_out || !(tol > 0) || max_iter < 1 || max_iter > 100000 || restart < 0)
    return ctx->fail(SESM_EINVAL, "bad solve arguments");
  SESM_HIP(hipSetDevice(ctx->device));
  const int N = ctx->P.N;
  int m = (restart == 0 || restart > max_iter) ? max_iter : restart;
  if (m > 4000) return ctx->fail(SESM_EINVAL, "Krylov dimension above 4000; use restart");
  int rc = ensure_workspace(ctx, m);
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  const int nb = (N + 255) / 256;
  cplx* x = (cplx*)mu_out;
  cplx* V = ctx->V;
  const int64_t ldv = N;
  double* npart = (double*)ctx->hpart;  // reuse for norm partials

  // right-hand side (incident field written into the workspace vector when NULL)
  const cplx* b = (const cplx*)b_in;
  if (!b) {
    if ((rc = sesm_rhs(ctx, (sesm_c64*)ctx->wtmp))) return rc;
    b = ctx->wtmp;
  }
  auto norm_to_host = [&](const cplx* v, double* out) -> int {
    hipLaunchKernelGGL(k_norm2_part, dim3(NCHUNK), dim3(256), 0, st, N, v, npart);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, npart, ctx->hcol);
    SESM_LAUNCH_CHECK();
    SESM_HIP(hipMemcpyAsync(ctx->hhost, ctx->hcol, sizeof(cplx), hipMemcpyDeviceToHost, st));
    SESM_HIP(hipStreamSynchronize(st));
    *out = ctx->hhost[0].re;
    return SESM_OK;
  };
  // Arnoldi step `it`: w = A v_it, CGS2 against v_0..v_it, normalise; the
  // column (h_0..h_it, |w|) goes to ring slot it % SESM_HRING, then to the host.
  auto arnoldi = [&](int it) -> int {
    cplx* w = V + (int64_t)(it + 1) * ldv;
    int r = sesm_apply(ctx, V + (int64_t)it * ldv, w);
    if (r) return r;
    const int nv = it + 1, slot = it % SESM_HRING;
    cplx* hc = ctx->hcol + (size_t)slot * SESM_HSTRIDE;
    const dim3 gd(DCHUNK, (nv + VT - 1) / VT);
    const int nch = (nv + UCH - 1) / UCH;
    const double c16 = sizeof(cplx);
    for (int pass = 0; pass < 2; ++pass) {
      SESM_KT_BEGIN(SESM_KT_DOTS, st);
      hipLaunchKernelGGL(k_dots, gd, dim3(256), 0, st, N, nv, V, ldv, w, ctx->hpart);
      SESM_KT_END(SESM_KT_DOTS, st, c16 * ((double)nv * N + N + (double)nv * DCHUNK));  // basis, w, partials
      SESM_KT_BEGIN(SESM_KT_UPDATE, st);
      hipLaunchKernelGGL(k_update_part, dim3(nb, nch), dim3(256), 0, st, N, nv, V, ldv, ctx->hpart, hc, pass,
                         ctx->upart);
      // basis, update partials, dot partials
      SESM_KT_END(SESM_KT_UPDATE, st, c16 * ((double)nv * N + (double)nch * N + (double)nv * DCHUNK));
      hipLaunchKernelGGL(k_update_final, dim3(nb), dim3(256), 0, st, N, nch, ctx->upart, w,
                         pass == 1 ? npart : nullptr);
    }
    hipLaunchKernelGGL(k_scale_norm, dim3(nb), dim3(256), 0, st, N, nb, npart, w, hc + nv);
    SESM_LAUNCH_CHECK();
    SESM_HIP(hipMemcpyAsync(ctx->hhost + (size_t)slot * SESM_HSTRIDE, hc, sizeof(cplx) * (nv + 1),
                            hipMemcpyDeviceToHost, st));
    SESM_HIP(hipEventRecord(ctx->hev[slot], st));
    return SESM_OK;
  };
  double bnorm = 0.0;
  if ((rc = norm_to_host(b, &bnorm))) return rc;
  SESM_HIP(hipMemsetAsync(x, 0, sizeof(cplx) * (size_t)N, st));
  sesm_solve_info inf{0, 0.0, 0};
  if (bnorm == 0.0) {
    inf.converged = 1;
    if (info) *info = inf;
    return SESM_OK;
  }
  std::vector<std::complex<double>> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  int total = 0;
  double res = 1.0;
  bool first = true;
  while (total < max_iter) {
    // r = b - A x  (x = 0 on the first cycle)
    double beta0;
    if (first) {
      SESM_HIP(hipMemcpyAsync(V, b, sizeof(cplx) * (size_t)N, hipMemcpyDeviceToDevice, st));
      first = false;
    } else {
      if ((rc = sesm_apply(ctx, x, V))) return rc;
      hipLaunchKernelGGL(k_sub_from, dim3(nb), dim3(256), 0, st, N, b, V);
      SESM_LAUNCH_CHECK();
    }
    if ((rc = norm_to_host(V, &beta0))) return rc;
    res = beta0 / bnorm;
    if (res <= tol) break;
    hipLaunchKernelGGL(k_scale, dim3(nb), dim3(256), 0, st, N, V, ctx->hcol, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta0;
    const int steps = std::min(m, max_iter - total);  // Arnoldi steps available in this cycle
    if ((rc = arnoldi(0))) return rc;
    int it = 0;
    for (; it < steps; ++it, ++total) {
      if (it + 1 < steps && (rc = arnoldi(it + 1))) return rc;  // keep the device one step ahead
      const int nv = it + 1, slot = it % SESM_HRING;
      SESM_HIP(hipEventSynchronize(ctx->hev[slot]));
      const cplx* hh = ctx->hhost + (size_t)slot * SESM_HSTRIDE;
      std::complex<double>* col = &H[(size_t)it * (m + 1)];
      for (int t = 0; t <= nv; ++t) col[t] = std::complex<double>(hh[t].re, hh[t].im);
      for (int t = 0; t < it; ++t) {  // previous rotations [[conj c, conj s], [-s, c]]
        const std::complex<double> u = col[t], v = col[t + 1];
        col[t] = std::conj(cs[t]) * u + std::conj(sn[t]) * v;
        col[t + 1] = -sn[t] * u + cs[t] * v;
      }
      const std::complex<double> a = col[it], bb = col[it + 1];
      const double r = std::sqrt(std::norm(a) + std::norm(bb));
      cs[it] = r != 0 ? a / r : 1.0;
      sn[it] = r != 0 ? bb / r : 0.0;
      col[it] = r;
      col[it + 1] = 0.0;
      g[it + 1] = -sn[it] * g[it];
      g[it] = std::conj(cs[it]) * g[it];
      res = std::abs(g[it + 1]) / bnorm;
      if (res <= tol || r == 0.0) {
        ++it;
        ++total;
        break;
      }
    }
    // y = R^{-1} g, x += V y  (a step enqueued ahead of a converged one only wrote
    // v_{it+1} and a ring slot; both are ignored)
    const int nv = it;
    std::vector<std::complex<double>> y(nv);
    for (int t = nv - 1; t >= 0; --t) {
      std::complex<double> s = g[t];
      for (int u = t + 1; u < nv; ++u) s -= H[(size_t)u * (m + 1) + t] * y[u];
      y[t] = s / H[(size_t)t * (m + 1) + t];
    }
    cplx* yh = ctx->hhost + (size_t)SESM_HRING * SESM_HSTRIDE;  // idle: each cycle ends synchronised
    for (int t = 0; t < nv; ++t) yh[t] = cplx{y[t].real(), y[t].imag()};
    SESM_HIP(hipMemcpyAsync(ctx->ybuf, yh, sizeof(cplx) * nv, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), sizeof(cplx) * nv, st, N, nv, V, ldv, ctx->ybuf, x, 1);
    SESM_LAUNCH_CHECK();
    SESM_HIP(hipStreamSynchronize(st));
    if (res <= tol) break;
  }
  inf.iters = total;
  inf.rel_residual = res;
  inf.converged = res <= tol ? 1 : 0;
  if (info) *info = inf;
  if (!inf.converged) return ctx->fail(SESM_ENOCONV, "GMRES did not reach the tolerance");
  return SESM_OK;
}
