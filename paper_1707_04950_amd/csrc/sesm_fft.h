// Own FP64 complex FFT for the periodic (x) direction of the equivalent-source
// grids: self-sorting mixed-radix (2, 3, 4, 5) Stockham transform, one row per
// 256-thread workgroup, both ping-pong buffers in LDS, twiddles from a table
// w[t] = exp(-2 pi i t / n) built on the host.  Rows are read and written with
// unit stride (coalesced).  Optional fused pre/post multiplication by
// exp(-/+ i alpha x) (the quasi-periodic twist) and 1/n scaling.
#pragma once
#include <vector>

#include "sesm_math.h"

#define SESM_FFT_MAXN 2000
#define SESM_FFT_MAXRAD 16

struct FftPlan {
  int n = 0, nrad = 0;
  int rad[SESM_FFT_MAXRAD];
  cplx* tw = nullptr;  // device table, length n
};

// Factor n into radices 4, 2, 3, 5 (in that order); false if another prime divides n.
inline bool sesm_fft_factor(int n, FftPlan* p) {
  p->n = n;
  p->nrad = 0;
  const int order[4] = {4, 2, 3, 5};
  for (int t = 0; t < 4; ++t) {
    while (n % order[t] == 0) {
      if (p->nrad >= SESM_FFT_MAXRAD) return false;
      p->rad[p->nrad++] = order[t];
      n /= order[t];
    }
  }
  return n == 1;
}

struct FftArgs {
  int n, nrad;
  int rad[SESM_FFT_MAXRAD];
};

// rows of `in` (row r at in + r*ld_in) -> rows of `out`; in-place allowed.
//   out = sign < 0 ? FFT(pre . in) : IFFT-like sum with e^{+}, then . post * scale
// pre/post: optional per-column factors (length n), may be null.
__global__ __launch_bounds__(256) void k_fft_rows(FftArgs A, const cplx* in, int64_t ld_in, cplx* out,
                                                  int64_t ld_out, const cplx* __restrict__ tw, int sign,
                                                  const cplx* __restrict__ pre, const cplx* __restrict__ post,
                                                  double scale) {
  __shared__ cplx buf[2][SESM_FFT_MAXN];
  const int n = A.n;
  const cplx* src = in + (int64_t)blockIdx.x * ld_in;
  cplx* a = buf[0];
  cplx* b = buf[1];
  for (int i = threadIdx.x; i < n; i += 256) {
    cplx v = src[i];
    if (pre) v = v * pre[i];
    a[i] = v;
  }
  __syncthreads();
  int p = 1;
  for (int s = 0; s < A.nrad; ++s) {
    const int R = A.rad[s];
    const int T = n / R;
    const int step = n / (p * R);  // twiddle stride for exp(-2 pi i q k / (p R))
    const int rstep = n / R;       // twiddle stride for the radix-R DFT
    for (int i = threadIdx.x; i < T; i += 256) {
      const int k = i % p;
      cplx x[5];
      for (int q = 0; q < R; ++q) {
        cplx w = tw[(q * k * step) % n];
        if (sign > 0) w = conj(w);
        x[q] = a[i + q * T] * w;
      }
      const int j = (i / p) * p * R + k;
      for (int u = 0; u < R; ++u) {
        cplx y = x[0];
        for (int q = 1; q < R; ++q) {
          cplx w = tw[((u * q) % R) * rstep];
          if (sign > 0) w = conj(w);
          y += x[q] * w;
        }
        b[j + u * p] = y;
      }
    }
    __syncthreads();
    cplx* t = a;
    a = b;
    b = t;
    p *= R;
  }
  cplx* dst = out + (int64_t)blockIdx.x * ld_out;
  for (int i = threadIdx.x; i < n; i += 256) {
    cplx v = scale * a[i];
    if (post) v = v * post[i];
    dst[i] = v;
  }
}

inline FftArgs sesm_fft_args(const FftPlan& p) {
  FftArgs A;
  A.n = p.n;
  A.nrad = p.nrad;
  for (int t = 0; t < SESM_FFT_MAXRAD; ++t) A.rad[t] = t < p.nrad ? p.rad[t] : 1;
  return A;
}
