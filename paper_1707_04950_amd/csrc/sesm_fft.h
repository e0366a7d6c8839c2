// Own FP64 complex FFT for the periodic (x) direction of the equivalent-source
// grids: self-sorting mixed-radix (2, 3, 4, 5) Stockham transform, one row per
// workgroup (several short rows share one; two grids may share a launch), both
// ping-pong buffers in LDS, twiddles from a table
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

// radices packed three bits each, pass s in bits 3s..3s+2 (kept free of
// arrays so that a job copied into registers needs no private memory)
struct FftArgs {
  int n, nrad;
  uint64_t radcode;
};

// Radix-R butterflies y_u = sum_q x_q w^{uq}, w = exp(sign 2 pi i / R).
__device__ inline void sesm_dft_small(int R, int sign, cplx* x) {
  const double sg = sign < 0 ? -1.0 : 1.0;
  if (R == 2) {
    const cplx a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  } else if (R == 4) {
    const cplx a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3], d = x[1] - x[3];
    const cplx id = sg * mul_i(d);  // sign * i * d
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + id;
    x[3] = b - id;
  } else if (R == 3) {
    const double c1 = -0.5, s1 = sg * 0.86602540378443864676;
    const cplx t = x[1] + x[2], u = x[1] - x[2];
    const cplx m = x[0] + c1 * t;
    const cplx iu = s1 * mul_i(u);
    x[0] = x[0] + t;
    x[1] = m + iu;
    x[2] = m - iu;
  } else {  // R == 5
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = sg * 0.95105651629515357212, s2 = sg * 0.58778525229247312917;
    const cplx t1 = x[1] + x[4], t2 = x[2] + x[3], u1 = x[1] - x[4], u2 = x[2] - x[3];
    const cplx a1 = x[0] + c1 * t1 + c2 * t2, a2 = x[0] + c2 * t1 + c1 * t2;
    const cplx b1 = mul_i(s1 * u1 + s2 * u2), b2 = mul_i(s2 * u1 - s1 * u2);
    x[0] = x[0] + t1 + t2;
    x[1] = a1 + b1;
    x[4] = a1 - b1;
    x[2] = a2 + b2;
    x[3] = a2 - b2;
  }
}

// One Stockham pass of radix R (a compile-time constant, so the butterfly
// operands stay in registers): p = product of the radices already applied,
// step = n / (p R) is the twiddle stride, exp(-2 pi i q k / (p R)) = tw[q k step].
template <int R>
__device__ inline void sesm_fft_pass(const cplx* a, cplx* b, int n, int nr, int p, int step,
                                     const cplx* __restrict__ tw, int sign) {
  const int T = n / R;
  for (int e = threadIdx.x; e < nr * T; e += blockDim.x) {
    const int r = e / T, i = e - r * T;
    const int k = i % p;
    const cplx* ar = a + r * n;
    cplx x[R];
    x[0] = ar[i];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      cplx w = tw[q * k * step];
      if (sign > 0) w = conj(w);
      x[q] = ar[i + q * T] * w;
    }
    sesm_dft_small(R, sign, x);
    cplx* br = b + r * n;
    const int j = (i - k) * R + k;  // (i / p) p R + k
#pragma unroll
    for (int u = 0; u < R; ++u) br[j + u * p] = x[u];
  }
}

// One batch of rows of one length: rpb rows of length n per workgroup, row r
// read from in + r n and written to out + r n (in-place allowed).
// out = scale * (DFT with exp(sign 2 pi i jk/n) of (pre . in)) . post;
// pre/post optional (length n).
struct FftJob {
  FftArgs A;
  int nrows, rpb, nblocks;
  const cplx* in;
  cplx* out;
  const cplx* tw;
  const cplx* pre;
  const cplx* post;
  double scale;
};

// Batched launches of two jobs: member blockIdx.y reads in + m bin and writes
// out + m bout of each job.
struct FftBatch {
  int64_t bin0, bout0, bin1, bout1;
  int64_t bpost0, bpost1;  // per-member offsets of each job's post factors (0: shared)
};

// The transform of one workgroup's rows of job J: the rows' elements come
// from load(row, col) (row of the job, column 0..n-1), two per thread in
// flight; the passes run in LDS; out = scale * transform . post.
template <class Loader>
__device__ inline void sesm_fft_block(const FftJob J, int blk, int sign, Loader load) {
  __shared__ cplx buf[2][SESM_FFT_MAXN];
  const int n = J.A.n;
  const int r0 = blk * J.rpb;
  const int nr = min(J.rpb, J.nrows - r0);
  const cplx* __restrict__ tw = J.tw;
  cplx* a = buf[0];
  cplx* b = buf[1];
  for (int e0 = threadIdx.x; e0 < nr * n; e0 += 2 * blockDim.x) {  // two elements in flight per thread
    cplx v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + u * (int)blockDim.x, nr * n - 1);
      v[u] = load(r0 + e / n, e % n);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < nr * n) a[e] = v[u];
    }
  }
  __syncthreads();
  int p = 1;
  for (int s = 0; s < J.A.nrad; ++s) {
    const int R = (int)((J.A.radcode >> (3 * s)) & 7u);
    const int step = n / (p * R);
    switch (R) {
      case 4: sesm_fft_pass<4>(a, b, n, nr, p, step, tw, sign); break;
      case 2: sesm_fft_pass<2>(a, b, n, nr, p, step, tw, sign); break;
      case 3: sesm_fft_pass<3>(a, b, n, nr, p, step, tw, sign); break;
      default: sesm_fft_pass<5>(a, b, n, nr, p, step, tw, sign); break;
    }
    __syncthreads();
    cplx* t = a;
    a = b;
    b = t;
    p *= R;
  }
  for (int e = threadIdx.x; e < nr * n; e += blockDim.x) {
    const int i = e % n;
    cplx v = J.scale * a[e];
    if (J.post) v = v * J.post[i];
    J.out[(int64_t)r0 * n + e] = v;
  }
}

// Workgroups [0, j0.nblocks) run job j0, the next j1.nblocks run job j1 (two
// grids of different lengths in one launch); rows read from in (times pre).
__global__ __launch_bounds__(1024) void k_fft_rows(FftJob j0, FftJob j1, int sign) {
  const bool first = (int)blockIdx.x < j0.nblocks;
  const FftJob J = first ? j0 : j1;
  const int blk = first ? blockIdx.x : blockIdx.x - j0.nblocks;
  const int n = J.A.n;
  const cplx* in = J.in;
  const cplx* pre = J.pre;
  sesm_fft_block(J, blk, sign, [=](int r, int i) {
    const cplx v = in[(int64_t)r * n + i];
    return pre ? v * pre[i] : v;
  });
}

// The same for several batch members: grid dimension y runs over them, member
// m reading in + m bin and writing out + m bout of its job (post factors at
// post + m bpost).
__global__ __launch_bounds__(1024) void k_fft_rows_batch(FftJob j0, FftJob j1, int sign, FftBatch fb) {
  const bool first = (int)blockIdx.x < j0.nblocks;
  FftJob J = first ? j0 : j1;
  const int64_t m = blockIdx.y;
  J.out += m * (first ? fb.bout0 : fb.bout1);
  if (J.post) J.post += m * (first ? fb.bpost0 : fb.bpost1);
  const int blk = first ? blockIdx.x : blockIdx.x - j0.nblocks;
  const int n = J.A.n;
  const cplx* in = J.in + m * (first ? fb.bin0 : fb.bin1);
  const cplx* pre = J.pre;
  sesm_fft_block(J, blk, sign, [=](int r, int i) {
    const cplx v = in[(int64_t)r * n + i];
    return pre ? v * pre[i] : v;
  });
}

inline FftArgs sesm_fft_args(const FftPlan& p) {
  FftArgs A;
  A.n = p.n;
  A.nrad = p.nrad;
  A.radcode = 0;
  for (int t = 0; t < p.nrad; ++t) A.radcode |= (uint64_t)p.rad[t] << (3 * t);
  return A;
}

// A job for `rows` rows of plan p (empty job when rows == 0).
inline FftJob sesm_fft_job(const FftPlan& p, int rows, const cplx* in, cplx* out, const cplx* pre, const cplx* post,
                           double scale) {
  FftJob J{};
  J.A = sesm_fft_args(p);
  J.nrows = rows;
  J.rpb = rows > 0 ? (p.n < SESM_FFT_MAXN ? SESM_FFT_MAXN / p.n : 1) : 1;
  if (J.rpb > rows && rows > 0) J.rpb = rows;
  J.nblocks = rows > 0 ? (rows + J.rpb - 1) / J.rpb : 0;
  J.in = in;
  J.out = out;
  J.tw = p.tw;
  J.pre = pre;
  J.post = post;
  J.scale = scale;
  return J;
}
