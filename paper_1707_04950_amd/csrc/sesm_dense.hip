// Dense direct operator (Sec. 4.3): assembly of (1/2 I + D^dx) and its GEMV.
//
// Entry (i, l) sums, over the images p of source l (x_l + p d, density phase
// e^{i alpha p d}, eq. quasiper_disc):
//   regular part   dx S_{cA,A}(X_p) (1 - S^f) K_dl          eq. (DAdx_def)
//   singular part  S^f (R_{l-i} K_s + dx K_r)                eq. (local_mat)
// with X_p = x_i - x_l - p d, Y = f_i - f_l and the double-layer kernel per
// unit dx'  K_dl = sum_m (-1)^m C(j,m) (ik/4) H1(k R_m) (Y + m h - f'_l X_p) / R_m;
// plus the completion modes D_M (eq. M_eta, trapezoidal rule) and 1/2 on the
// diagonal, where D~_sing contributes dx K_r(x,x).
//
// One 64-lane wavefront per matrix entry, lanes over lattice images p, a
// DPP/shuffle reduction at the end: the windowed lattice sum is the FP64-heavy
// part (up to (2A+3)(j+1) Hankel evaluations per entry).
#include "sesm_kernels.h"

namespace {

__global__ __launch_bounds__(256) void k_dense_assemble(KParams K, const double* __restrict__ x,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ fp,
                                                        const double* __restrict__ fpp,
                                                        const double* __restrict__ J,
                                                        const double* __restrict__ logw, cplx* __restrict__ M) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y;                             // row (target node)
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);    // column (source node), one per wave
  if (l >= K.N) return;  // wave-uniform
  const int64_t e = (int64_t)i * K.N + l;
  const double X0 = x[i] - x[l], Y = f[i] - f[l], fps = fp[l];
  cplx acc = cplx{0.0, 0.0};
  for (int p = K.pmin + lane; p <= K.pmax; p += 64) {
    const double Xp = X0 - p * K.d;
    const double SA = sesm_window(Xp, K.cA, K.A_len);
    if (SA == 0.0) continue;
    if (p == 0 && i == l) continue;  // diagonal: handled below
    acc += cexp_i(K.alpha * p * K.d) * sesm_entry_offdiag(K, logw, Xp, Y, fps, SA);
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    if (i == l) acc += sesm_entry_diag(K, fp[i], fpp[i]);
    for (int t = 0; t < K.nU; ++t) {
      const double mag = exp(-K.Ubi[t] * Y);
      acc += (mag * J[l] * K.dx) * cexp_i(K.Ua[t] * X0 + K.Ubr[t] * Y);
    }
    M[e] = acc;
  }
}

// y_i = sum_l M_il mu_l: one 256-thread block per row (the operator streamed
// past the caches, which keep the Krylov basis).
__global__ __launch_bounds__(256) void k_gemv_rows(int N, const cplx* __restrict__ M, const cplx* __restrict__ mu,
                                                   cplx* __restrict__ y) {
  __shared__ cplx sh[4];
  const cplx* row = M + (int64_t)blockIdx.x * N;
  cplx acc = cplx{0.0, 0.0};
  for (int l = threadIdx.x; l < N; l += 256) acc += load_stream(&row[l]) * mu[l];
  const cplx s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) y[blockIdx.x] = s;
}

}  // namespace

int sesm_dense_setup(sesm_ctx* ctx) {
  const Problem& P = ctx->P;
  const int64_t NN = (int64_t)P.N * P.N;
  int rc = sesm_alloc(ctx, (void**)&ctx->Mdense, sizeof(cplx) * (size_t)NN);
  if (rc) return rc;
  const KParams K = ctx->kparams();
  if (P.N > 65535) return ctx->fail(SESM_EINVAL, "dense mode supports N <= 65535");
  if (ctx->prm.adjoint == 1) return sesm_dense_assemble_with_derivs(ctx);
  hipLaunchKernelGGL(k_dense_assemble, dim3((P.N + 3) / 4, P.N), dim3(256), 0, ctx->stream, K, ctx->x, ctx->f, ctx->fp,
                     ctx->fpp, ctx->J, ctx->logw, ctx->Mdense);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

int sesm_dense_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y) {
  if (ctx->adjoint) return sesm_dense_matvec_adjoint(ctx, mu, y);
  const double N = ctx->P.N;
  SESM_KT_BEGIN(SESM_KT_GEMV, ctx->stream);
  hipLaunchKernelGGL(k_gemv_rows, dim3(ctx->P.N), dim3(256), 0, ctx->stream, ctx->P.N, ctx->Mdense, mu, y);
  SESM_LAUNCH_CHECK();
  SESM_KT_END(SESM_KT_GEMV, ctx->stream, sizeof(cplx) * (N * N + 2.0 * N));  // operator, mu, y
  return SESM_OK;
}
