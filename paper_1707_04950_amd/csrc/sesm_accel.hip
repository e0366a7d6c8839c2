// Shifted-equivalent-source FFT accelerator (Sec. 5; Algorithms 2 and 3).
//
// Geometry: square cells of side L = d / n_x (n_x 5-smooth, >= 3), half-open
// (a1,b1] x (a2,b2] (Remark cell_def), columns from x0 = -dx/2, rows from y0
// below the surface to y0 + n_y L above it.  Equivalent-source grid spacing
// delta = L / n_s; each cell carries a horizontal set (bottom and top sides)
// and a vertical set (left and right sides), each side extended by n_e grid
// points beyond the corners (eq. eq_mesh), monopoles plus dipoles with the
// fixed normals (0,1) / (1,0) so that densities of neighbouring cells add at
// shared grid points (eq. sum_eqsources).
//
// Near/far split: the near (direct) set of a target cell is every source of
// the 2 ring + 1 columns around it (ring = 1 by default) - a superset of the
// paper's intersecting cells
// L(q) (eq. small_convolution); all other cells are non-intersecting because
// the target cell lies outside their 3L squares and all downward shifts
// (eq. S_jq_hat).  On a graph surface the near set of a column is one cyclic
// band of nodes, stored as dense FP64 blocks (the HBM-bound part).
//
// Forward map, one stream, in order:
//   k_local_apply   y  = near band (intersecting part eq. final_correction_0,
//                        singular part eq. local_mat, 1/2 I);
//                   (xi, zeta)^{q,lambda} = P_q^lambda mu_q   (EqSources, eq. eq_source_point);
//                   partial sums of the completion modes      (EvalModes, eq. M_eta)
//   k_merge_fft     twisted merged grids, gathered straight into the FFT along x
//                   of both grids                            (GlobalEqSMerge, eq. sum_eqsources;
//                                                             GlobalFFT, eq. large_convolution_per_grid)
//   k_yconv         kernel-spectrum x sources, direct in y
//                   + local corrections per cell pair         (LocalEqSMerge, LocalFFT, eq. small_convolution)
//   k_fft_rows      inverse FFT, untwist -> phi^all
//   k_cells_far     boundary values - local corrections       (LocalSubtract, Combine-lambda,
//                   -> plane-wave weights -> surface values      PlaneWaveWeights, NonIntersecting;
//                   + completion modes D_M, added into y         eqs. psi_na_sum, combine_psi_pna,
//                                                                planewave, plwave_QR)
// The near field and the equivalent-source densities share one launch: both
// stream stored operators from HBM and depend on mu only, while the grid
// stages after them are latency-bound and would slow down beside a stream.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

#include "sesm_fft.h"
#include "sesm_kernels.h"

using C = std::complex<double>;

struct AccelOp {
  // geometry
  int n_x = 0, n_y = 0, n_s = 0, n_e = 0, n_coll = 0, n_plw = 0, ring = 1;
  int n_side = 0, n_eq = 0, n_bH = 0, n_bdry = 0, n_cells = 0, n_occ = 0, n_off = 0;
  int max_q = 0;  // most nodes in one occupied cell
  double L = 0, delta = 0, x0 = 0, y0 = 0;
  int nXH = 0, nYH = 0, nXV = 0, nYV = 0;
  int64_t near_entries = 0;
  // device data
  int *occ_cell = nullptr, *occ_off = nullptr, *perm = nullptr, *col_lo = nullptr, *col_w = nullptr;
  int64_t* near_off = nullptr;
  int n_chunks = 0, max_w = 0;  // near-field row chunks (cell, first row); widest band
  int *chunk_q = nullptr, *chunk_t0 = nullptr;
  int n_cfc = 0;  // far-field work items: up to CF_NODES nodes of one cell (cell, first node)
  int *cfc_q = nullptr, *cfc_t0 = nullptr;
  cplx *p2e = nullptr, *nearblk = nullptr, *dens = nullptr;
  cplxf* p2e32 = nullptr;  // the EqSources operators in FP32 (mixed-precision map; built on request)
  cplx *gH = nullptr, *gV = nullptr, *fH = nullptr, *fV = nullptr, *phH = nullptr, *phV = nullptr;
  cplx *specH = nullptr, *specV = nullptr, *W = nullptr;  // (inside self_spec)
  cplx *pplw = nullptr;  // plane-wave least squares: (U^H)^T (n_bdry x n_plw), V^T (n_plw x n_plw), 1 / sig
  cplx *pinv = nullptr;  // equivalent-source least squares, per set: Q^H (2n_eq x 4n_coll) then R
  cplx *twxH = nullptr, *twxV = nullptr, *utwH = nullptr, *utwV = nullptr;  // e^{-i alpha x}, e^{+i alpha x} (inside self_tw)
  double* dirs = nullptr;
  cplx* mode_part = nullptr;
  // local-correction pairs (occupied cell q, occupied cell of its near columns):
  // pair_off[q]..pair_off[q+1]-1, correction-matrix offset, source cell, wrap phase
  int n_pairs = 0, n_groups = 0;
  int* pair_off = nullptr;
  int *grp_o = nullptr, *grp_start = nullptr, *grp_n = nullptr, *plist = nullptr;  // pairs grouped by offset
  int* grp_rc = nullptr;   // source cell per pair, in plist order

  cplx* corr = nullptr;  // [n_pairs][n_bdry]
  cplx* yfar = nullptr;  // diagnostic copy of the far-field contribution
  cplx* bq = nullptr;    // diagnostic copy of the boundary values b^q, [n_occ][n_bdry]
  // batched forward maps: the per-density work buffers of up to kBatchMax
  // densities (allocated at the first batched call)
  cplx* batch_ws = nullptr;
  FftPlan planH, planV;
  // near-field items of a single-density forward map: [0, c1) in the first
  // launch, [c1, c2) with merge + FFT, [c2, c3) with the y convolution,
  // [c3, n_chunks) with the inverse FFT (chosen by the tuner or the caller)
  int near_c1 = 0, near_c2 = 0, near_c3 = 0;
  double tuned_us = 0.0;                  // forward-map time of the chosen split (0: not measured)
  std::vector<int64_t> item_entries;      // prefix sums over the items: stored entries
  std::vector<int64_t> item_rows;         //                              rows
  // incidence-dependent tables, laid out alike for the surface's own
  // incidence and for each member of an incidence set: kernel spectra
  // [specH | specV] (spec_len entries) and twist factors
  // [e^{-i alpha x} on H | on V | e^{+i alpha x} on H | on V] (tw_len entries)
  int64_t spec_len = 0, tw_len = 0;
  cplx *self_spec = nullptr, *self_tw = nullptr;
  // hybrid tables (Sec. 3.2): per grid, the rows taken by the windowed sums and
  // the rows taken by the spectral series with their truncation orders
  struct HybridRows {
    std::vector<int> spatial, spectral, nmax;
    int *d_spatial = nullptr, *d_spectral = nullptr, *d_nmax = nullptr;
  } hyb[2];
  bool hybrid = false;
  // batched near field on the matrix cores: 16-row tiles (cell, first row)
  bool batch_mfma = false;
  int n_tiles = 0;
  int *tile_q = nullptr, *tile_t0 = nullptr;
  IncParams* inc_self = nullptr;          // device record of the surface's incidence
  int n_inc = 0;                          // incidence set (sesm_set_incidences)
  IncParams* inc_set = nullptr;           // device records [n_inc]
  cplx *inc_spec = nullptr, *inc_tw = nullptr;
  std::vector<Problem> inc_prob;          // each member's incidence-dependent scalars (host)
  int* grp_wr = nullptr;                  // column wrap of each correction pair's source cell
};

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr int NCH_MODES = 240;
constexpr int kBatchMax = 4;  // densities per batched local launch
constexpr int CF_NODES = 64;  // nodes per workgroup of the cell far-field kernel

int smooth5_at_least(int n) {
  for (;; ++n) {
    int m = n;
    for (int p : {2, 3, 5})
      while (m % p == 0) m /= p;
    if (m == 1) return n;
  }
}

// Least squares by Householder QR (the "QR-based solution" of eqs.
// eq_source_point and plwave_QR): factors the m x n matrix A (row-major,
// m >= n) as A = Q R and returns the first n rows of Q^H (n x m) and the upper
// triangle R (n x n), both row-major.  Solutions are then obtained by
// back-substitution R x = Q^H b for each right-hand side, never through an
// explicit pseudo-inverse (which loses the small residual when A is
// ill-conditioned).  False if A is rank deficient.
bool ls_qr(int m, int n, std::vector<C> A, std::vector<C>& Qh_out, std::vector<C>& R_out) {
  // plain complex products (finite operands), so that the loops stay inline
  auto mul = [](C a, C b) { return C(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real()); };
  auto cmul = [](C a, C b) {  // conj(a) b
    return C(a.real() * b.real() + a.imag() * b.imag(), a.real() * b.imag() - a.imag() * b.real());
  };
  std::vector<std::vector<C>> V(n);
  std::vector<C> colk(m);
  for (int k = 0; k < n; ++k) {
    double nx = 0;
    for (int i = k; i < m; ++i) nx += std::norm(A[(size_t)i * n + k]);
    nx = std::sqrt(nx);
    if (!(nx > 0)) return false;
    const C x0 = A[(size_t)k * n + k];
    const C ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : C(1.0, 0.0);
    const C alpha = -ph * nx;
    std::vector<C> v(m - k);
    for (int i = k; i < m; ++i) v[i - k] = A[(size_t)i * n + k];
    v[0] -= alpha;
    double vn = 0;
    for (const C& t : v) vn += std::norm(t);
    vn = std::sqrt(vn);
    for (C& t : v) t /= vn;
    // columns k..n-1 of the row-major A: one sweep over the rows accumulates
    // all their projections (independent sums), a second applies the update
    std::vector<C> sc(n - k, C(0.0));
    for (int i = k; i < m; ++i) {
      const C vi = v[i - k];
      const C* ar = &A[(size_t)i * n];
      for (int c = k; c < n; ++c) sc[c - k] += cmul(vi, ar[c]);
    }
    for (C& t : sc) t *= 2.0;
    for (int i = k; i < m; ++i) {
      const C vi = v[i - k];
      C* ar = &A[(size_t)i * n];
      for (int c = k; c < n; ++c) ar[c] -= mul(vi, sc[c - k]);
    }
    V[k] = std::move(v);
  }
  // the first n columns of Q = H_0 H_1 ... H_{n-1} (reflectors applied to
  // the identity's columns, last reflector first), stored column by column;
  // rows 0..n-1 of Q^H are their conjugates
  std::vector<C> Qc((size_t)n * m, 0.0);
  for (int c = 0; c < n; ++c) Qc[(size_t)c * m + c] = 1.0;
  for (int k = n - 1; k >= 0; --k) {
    const std::vector<C>& v = V[k];
    for (int c0 = 0; c0 < n; c0 += 4) {  // four columns at a time: independent sums
      const int nc = std::min(4, n - c0);
      C s[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = k; i < m; ++i)
        for (int u = 0; u < nc; ++u) s[u] += cmul(v[i - k], Qc[(size_t)(c0 + u) * m + i]);
      for (int u = 0; u < nc; ++u) {
        C* q = &Qc[(size_t)(c0 + u) * m];
        const C t = 2.0 * s[u];
        for (int i = k; i < m; ++i) q[i] -= mul(v[i - k], t);
      }
    }
  }
  Qh_out.resize((size_t)n * m);
  for (size_t t = 0; t < Qh_out.size(); ++t) Qh_out[t] = std::conj(Qc[t]);
  R_out.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    if (std::abs(A[(size_t)r * n + r]) == 0) return false;
    for (int c = r; c < n; ++c) R_out[(size_t)r * n + c] = A[(size_t)r * n + c];
  }
  return true;
}

// Singular value decomposition A = U diag(sig) V^H of an m x n matrix
// (used for the plane-wave least squares of eq. plwave_QR)
// (row-major, m >= n) by one-sided Jacobi rotations (Hestenes' method): pairs
// of columns are rotated until all are mutually orthogonal; the column norms
// are then the singular values, the normalised columns U, and the
// accumulated rotations V.  Least squares then reads w = V diag(1/sig) U^H b,
// applied factor by factor (stable like the QR route; the product of the
// factors is never formed).  Returns U^H (n x m, row-major), sig (n) and V
// (n x n, row-major).  False if a column vanishes (rank deficiency) or the
// sweeps do not converge.
bool ls_svd(int m, int n, const std::vector<C>& A, std::vector<C>& Uh_out, std::vector<double>& sig,
            std::vector<C>& V_out) {
  std::vector<C> a((size_t)n * m), v((size_t)n * n, C(0.0));  // column-major copies
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)j * m + i] = A[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) v[(size_t)j * n + j] = 1.0;
  bool converged = false;
  for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        C* ap = &a[(size_t)p * m];
        C* aq = &a[(size_t)q * m];
        double al = 0.0, be = 0.0;
        C ga = 0.0;
        for (int i = 0; i < m; ++i) {
          al += std::norm(ap[i]);
          be += std::norm(aq[i]);
          ga += std::conj(ap[i]) * aq[i];
        }
        const double g = std::abs(ga);
        if (!(g > 0.0) || g <= 1e-15 * std::sqrt(al * be)) continue;
        off = std::max(off, g / std::sqrt(al * be));
        const C e = std::conj(ga / g);  // aq e makes the pair's inner product real and positive
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const C x = ap[i], y = aq[i] * e;
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        C* vp = &v[(size_t)p * n];
        C* vq = &v[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const C x = vp[i], y = vq[i] * e;
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    converged = off <= 1e-15;
  }
  if (!converged) return false;
  sig.assign(n, 0.0);
  Uh_out.assign((size_t)n * m, C(0.0));
  V_out.assign((size_t)n * n, C(0.0));
  for (int j = 0; j < n; ++j) {
    double nn = 0.0;
    for (int i = 0; i < m; ++i) nn += std::norm(a[(size_t)j * m + i]);
    sig[j] = std::sqrt(nn);
    if (!(sig[j] > 0.0)) return false;
    for (int i = 0; i < m; ++i) Uh_out[(size_t)j * m + i] = std::conj(a[(size_t)j * m + i]) / sig[j];
    for (int i = 0; i < n; ++i) V_out[(size_t)i * n + j] = v[(size_t)j * n + i];
  }
  return true;
}

// Geometry of one cell, relative to its lower-left corner (all integer-indexed).
struct CellGeo {
  int n_s, n_e, n_side, n_eq, n_coll;
  double L, delta;
  // equivalent-source point s of set lam (0 = H, 1 = V)
  __host__ __device__ void eq_point(int lam, int s, double* px, double* py) const {
    const int side = s / n_side, i = s % n_side - n_e;
    if (lam == 0) {
      *px = i * delta;
      *py = side * L;
    } else {
      *px = side * L;
      *py = i * delta;
    }
  }
  // collocation point c on the boundary of the 3L square (n_coll per side)
  __host__ __device__ void coll_point(int c, double* px, double* py) const {
    const int side = c / n_coll, i = c % n_coll;
    const double t = (i + 0.5) / n_coll * 3.0 * L - L;
    if (side == 0) { *px = t; *py = -L; }
    else if (side == 1) { *px = t; *py = 2.0 * L; }
    else if (side == 2) { *px = -L; *py = t; }
    else { *px = 2.0 * L; *py = t; }
  }
  // boundary point b: horizontal sides first (corners included), then vertical sides
  __host__ __device__ void bdry_point(int b, double* px, double* py) const {
    const int nh = 2 * (n_s + 1);
    if (b < nh) {
      const int iy = b / (n_s + 1), i = b % (n_s + 1);
      *px = i * delta;
      *py = iy * L;
    } else {
      const int t = b - nh, ix = t / (n_s - 1), i = 1 + t % (n_s - 1);
      *px = ix * L;
      *py = i * delta;
    }
  }
};

// Back-substitution R x = y on one wavefront (n <= 64): lane u holds y_u on
// entry and x_u on exit; R upper triangular (n x n) stored column-major,
// R[u][r] at Rc[r n + u], so that the lanes' reads of a column are contiguous.
// Column-oriented: x_r is broadcast and subtracted from the rows above it.
__device__ inline cplx sesm_wave_backsub(const cplx* __restrict__ Rc, int n, cplx yu) {
  const int lane = threadIdx.x & 63;
  for (int r = n - 1; r >= 0; --r) {
    cplx xr = cplx{0.0, 0.0};
    if (lane == r) {
      const cplx d = Rc[(int64_t)r * n + r];
      const double dd = 1.0 / abs2(d);
      xr = cplx{(yu.re * d.re + yu.im * d.im) * dd, (yu.im * d.re - yu.re * d.im) * dd};
      yu = xr;
    }
    xr.re = sesm_readlane(xr.re, r);
    xr.im = sesm_readlane(xr.im, r);
    if (lane < r) yu -= Rc[(int64_t)r * n + lane] * xr;
  }
  return yu;
}


// sum over shifts of one free-space kernel between x and y, punctured term by
// term (terms with R_m <= 1e-9 h are dropped: the reading of eq. phi_def).
// kind 0: monopole Phi_j; 1: d/dy2 Phi_j (H dipole); 2: d/dy1 Phi_j (V dipole).
__device__ inline void sesm_green_pair(const KParams& K, int j, double X, double Y, cplx* mono, cplx* dip, int dkind) {
  cplx sm = cplx{0.0, 0.0}, sd = cplx{0.0, 0.0};
  const double thr = 1e-9 * (K.h > 0 ? K.h : 1.0);
  for (int m = 0; m <= j; ++m) {
    const double Ym = Y + m * K.h;
    const double R = sqrt(X * X + Ym * Ym);
    if (R <= thr) continue;
    cplx H0, H1;
    sesm_hankel01(K.k * R, &H0, &H1);
    const double w = (j == 0) ? 1.0 : K.wshift[m];
    sm += w * H0;
    sd += (w * (dkind == 1 ? Ym : X) / R) * H1;
  }
  *mono = 0.25 * mul_i(sm);
  *dip = (0.25 * K.k) * mul_i(sd);
}

// ------------------------------------------------------------------ setup kernels
// A_eq of eq. (eq_source_point): rows = collocation points, columns = monopoles then dipoles.
__global__ void k_aeq(KParams K, CellGeo G, int lam, cplx* A) {
  const int ncol = 2 * G.n_eq, nrow = 4 * G.n_coll;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrow * G.n_eq) return;
  const int r = e / G.n_eq, s = e % G.n_eq;
  double cx, cy, sx, sy;
  G.coll_point(r, &cx, &cy);
  G.eq_point(lam, s, &sx, &sy);
  cplx mono, dip;
  sesm_green_pair(K, 0, cx - sx, cy - sy, &mono, &dip, lam == 0 ? 1 : 2);
  A[(size_t)r * ncol + s] = mono;
  A[(size_t)r * ncol + G.n_eq + s] = dip;
}

// P_q = A_eq^+ B_q by QR: for every node l of the cell, B[:, l] holds the
// field of its surface true source at the collocation points,
// B[c][l] = dx (ik/4) H1(kR) (Y - f'_l X)/R (eq. true_field), and column l of
// P_q solves R x = Q^H B[:, l] (eq. eq_source_point), separately for the
// horizontal and the vertical set.  qr holds, per set, Q^H (ncol x nrow) then
// R (ncol x ncol), row-major.
__global__ __launch_bounds__(256) void k_p2e_setup(KParams K, CellGeo G, double x0, double y0, int n_x,
                                                   const int* __restrict__ chunk_q, const int* __restrict__ chunk_t0,
                                                   int rows_per_chunk,
                                                   const int* __restrict__ occ_cell, const int* __restrict__ occ_off,
                                                   const int* __restrict__ perm, const double* __restrict__ x,
                                                   const double* __restrict__ f, const double* __restrict__ fp,
                                                   const cplx* __restrict__ qr, cplx* __restrict__ P) {
  extern __shared__ cplx sh[];  // per wave: B (nrow)
  // one workgroup per chunk of up to rows_per_chunk nodes of one cell, one node per wavefront at a time
  const int q = chunk_q[blockIdx.x], c0 = chunk_t0[blockIdx.x];
  const int cell = occ_cell[q];
  const double ox = x0 + (cell % n_x) * G.L, oy = y0 + (cell / n_x) * G.L;
  const int off = occ_off[q], nq = occ_off[q + 1] - off;
  const int c1 = min(nq, c0 + rows_per_chunk);
  const int nrow = 4 * G.n_coll, ncol = 2 * G.n_eq;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cplx* B = sh + wv * nrow;
  cplx* Pq = P + (int64_t)2 * ncol * off;
  const int64_t per_set = (int64_t)ncol * nrow + (int64_t)ncol * ncol;
  for (int t0 = c0; t0 < c1; t0 += 4) {  // uniform trip count: barriers below are block-wide
    const int t = t0 + wv;
    if (t < c1) {
      const int l = perm[off + t];
      for (int c = lane; c < nrow; c += 64) {
        double cx, cy;
        G.coll_point(c, &cx, &cy);
        const double X = ox + cx - x[l], Y = oy + cy - f[l];
        const double R = sqrt(X * X + Y * Y);
        B[c] = (K.dx * 0.25 * K.k * (Y - fp[l] * X) / R) * mul_i(sesm_hankel1(K.k * R));
      }
    }
    __syncthreads();
    for (int lam = 0; lam < 2; ++lam) {  // ncol <= 64: one output row per lane
      const cplx* Qh = qr + lam * per_set;
      const cplx* Rm = Qh + (int64_t)ncol * nrow;
      if (t < c1) {
        cplx yu = cplx{0.0, 0.0};
        if (lane < ncol) {  // Q^H B: sixteen loads in flight, each a contiguous row of (Q^H)^T
          const cplx* qcol = Qh + lane;
          int c = 0;
          for (; c + 16 <= nrow; c += 16) {
            cplx qv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) qv[u] = qcol[(int64_t)(c + u) * ncol];
#pragma unroll
            for (int u = 0; u < 16; ++u) yu = cmac(yu, qv[u], B[c + u]);
          }
          for (; c < nrow; ++c) yu = cmac(yu, qcol[(int64_t)c * ncol], B[c]);
        }
        yu = sesm_wave_backsub(Rm, ncol, yu);
        if (lane < ncol) Pq[(int64_t)t * 2 * ncol + lam * ncol + lane] = yu;
      }
    }
    __syncthreads();
  }
}

// dst = src rounded to FP32 (n complex values)
__global__ void k_narrow(int64_t n, const cplx* __restrict__ src, cplxf* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = narrow_to<cplxf>(src[i]);
}

// Windowed lattice sums (eq. Gq_limit with the Bloch phase) of the monopole and
// dipole kernels on the difference grid, twisted by exp(-i alpha X):
// tab[kind][row][mx], row = my + nY - 1.  One wavefront per entry, lanes over images.
// rowmap (nullable): the rows to fill, nmap of them (otherwise all 2 nY - 1).
__global__ __launch_bounds__(256) void k_lattice(KParams K, int lam, int nX, int nY, double hx, double hy, int pmax,
                                                 const int* __restrict__ rowmap, int nmap, cplx* __restrict__ tab) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nrow = 2 * nY - 1;
  if (e >= (int64_t)nmap * nX) return;
  const int row = rowmap ? rowmap[e / nX] : (int)(e / nX), mx = (int)(e % nX);
  const double X = mx * hx, Y = (row - (nY - 1)) * hy;
  cplx sm = cplx{0.0, 0.0}, sd = cplx{0.0, 0.0};
  for (int p = -pmax + lane; p <= pmax; p += 64) {
    const double Xp = X + p * K.d;
    const double S = sesm_window(Xp, K.cA, K.A_len);
    if (S == 0.0) continue;
    cplx mono, dip;
    sesm_green_pair(K, K.j, Xp, Y, &mono, &dip, lam == 0 ? 1 : 2);
    const cplx ph = S * cexp_i(-K.alpha * K.d * p);
    sm += ph * mono;
    sd += ph * dip;
  }
  sm = wave_sum(sm);
  sd = wave_sum(sd);
  if (lane == 0) {
    const cplx tw = cexp_i(-K.alpha * X);
    tab[(int64_t)row * nX + mx] = sm * tw;
    tab[(int64_t)(nrow + row) * nX + mx] = sd * tw;
  }
}

// ---- hybrid tables: the spectral series of G~_j (Sec. 3.2)

__device__ inline cplx cdiv(cplx a, cplx b) { return (1.0 / abs2(b)) * cmul_conj(b, a); }
__device__ inline cplx cexp_iz(cplx z) {  // e^{i z}, z complex
  double sn, cs;
  sincos(z.re, &sn, &cs);
  const double m = exp(-z.im);
  return cplx{m * cs, m * sn};
}
__device__ inline cplx csin(cplx z) {
  double sn, cs;
  sincos(z.re, &sn, &cs);
  return cplx{sn * cosh(z.im), cs * sinh(z.im)};
}
__device__ inline cplx csinc(cplx z) {  // sin(z) / z
  if (abs2(z) < 1e-6) {
    const cplx z2 = z * z;
    return cplx{1.0, 0.0} - (1.0 / 6.0) * z2 + (1.0 / 120.0) * (z2 * z2);
  }
  return cdiv(csin(z), z);
}

// The y-dependence of mode n of the spectral series of G~_j (eq.
// shifted_quasi_per_rayleigh) at height Y, with t_m = Y + m h:
//   sb = sum_m w_m e^{i beta |t_m|} / beta,   sd = sum_m w_m sgn(t_m) e^{i beta |t_m|}.
// For |beta| < 1/2 (at and around Wood anomalies) sb takes the form of eq.
// betan_taylor with its beta-quotients written as limits-safe products:
//   e^{i beta Y} (1 - e^{i beta h})^j / beta
//     = e^{i beta (Y + j h / 2)} (-2i)^j sin^{j-1}(beta h / 2) (h / 2) sinc(beta h / 2),
//   (e^{i beta t} - e^{-i beta t}) / beta = 2 i t sinc(beta t)   (the rows t_m < 0).
// Needs j >= 1.
__device__ inline void spectral_y_sums(const KParams& K, cplx beta, double Y, cplx* sb, cplx* sd) {
  cplx b_ = cplx{0.0, 0.0}, d_ = cplx{0.0, 0.0};
  const bool small = abs2(beta) < 0.25;  // (the closed form grows like e^{|Im beta| |Y|} for evanescent terms)
  for (int m = 0; m <= K.j; ++m) {
    const double t = Y + m * K.h, at = fabs(t);
    const cplx e = cexp_iz(at * beta);
    d_ += (t < 0.0 ? -K.wshift[m] : K.wshift[m]) * e;
    if (!small) b_ += K.wshift[m] * e;
    else if (t < 0.0) b_ -= (2.0 * K.wshift[m] * t) * mul_i(csinc(t * beta));
  }
  if (small) {
    const cplx half = (0.5 * K.h) * beta;
    const cplx sh = csin(half);
    cplx pw = (0.5 * K.h) * csinc(half);
    for (int m = 1; m < K.j; ++m) pw = pw * sh;
    cplx c2 = cplx{1.0, 0.0};  // (-2i)^j
    for (int m = 0; m < K.j; ++m) c2 = cplx{2.0 * c2.im, -2.0 * c2.re};
    b_ += cexp_iz((Y + 0.5 * K.j * K.h) * beta) * (c2 * pw);
  } else {
    b_ = cdiv(b_, beta);
  }
  *sb = b_;
  *sd = d_;
}

// Spectral rows of the hybrid tables.  With X = mx d / nX on the periodic
// grid, G~_j e^{-i alpha X} = sum_n c_n e^{2 pi i n mx / nX}, so the x-transform
// of a table row is spec[b] = nX sum_{n = b (mod nX), |n| <= nmax} c_n, with
//   monopole c_n = (i / 2d) sb,  H dipole (d/dy2) c_n = (1 / 2d) sd,
//   V dipole (d/dx2) c_n = (alpha_n / 2d) sb.
// One workgroup per listed row (row r with truncation order nmax[r]);
// threads over the bins b; the terms of a bin are added in increasing n.
__global__ __launch_bounds__(256) void k_spectral_rows(KParams K, int lam, int nX, int nY, double hy,
                                                       const int* __restrict__ rows, const int* __restrict__ nmax,
                                                       cplx* __restrict__ spec) {
  const int row = rows[blockIdx.x], nm = nmax[blockIdx.x];
  const int nrow = 2 * nY - 1;
  const double Y = (row - (nY - 1)) * hy;
  const double inv2d = 0.5 / K.d, kk = K.k;
  for (int b = threadIdx.x; b < nX; b += blockDim.x) {
    const int qlo = -((nm + b) / nX);
    const int qhi = nm >= b ? (nm - b) / nX : -((b - nm + nX - 1) / nX);
    cplx am = cplx{0.0, 0.0}, ad = cplx{0.0, 0.0};
    for (int q = qlo; q <= qhi; ++q) {
      const int n = b + q * nX;
      const double an = K.alpha + 2.0 * SESM_PI * n / K.d;
      const double g = (kk - an) * (kk + an);
      const cplx beta = g >= 0.0 ? cplx{sqrt(g), 0.0} : cplx{0.0, sqrt(-g)};
      cplx sb, sd;
      spectral_y_sums(K, beta, Y, &sb, &sd);
      am += mul_i(inv2d * sb);
      ad += lam == 0 ? inv2d * sd : (an * inv2d) * sb;
    }
    spec[(int64_t)row * nX + b] = (double)nX * am;
    spec[(int64_t)(nrow + row) * nX + b] = (double)nX * ad;
  }
}

// Local-correction matrices W[o][s][b] (boundary point fastest): free-space
// punctured kernel from the equivalent sources of the cell at offset
// o = (ox, oy) to the boundary points of the cell at the origin (eq. small_convolution).
__global__ void k_wmat(KParams K, CellGeo G, int n_y, int ring, cplx* __restrict__ W) {
  const int nb = 2 * (G.n_s + 1) + 2 * (G.n_s - 1), ns2 = 2 * G.n_eq;
  const int noff = (2 * ring + 1) * (2 * n_y - 1);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)noff * nb * G.n_eq) return;
  const int s = (int)(e % G.n_eq);
  const int b = (int)((e / G.n_eq) % nb);
  const int o = (int)(e / ((int64_t)G.n_eq * nb));
  const int oxi = o / (2 * n_y - 1) - ring, oyi = o % (2 * n_y - 1) - (n_y - 1);
  const int lam = b < 2 * (G.n_s + 1) ? 0 : 1;
  double bx, by, sx, sy;
  G.bdry_point(b, &bx, &by);
  G.eq_point(lam, s, &sx, &sy);
  const double X = bx - (oxi * G.L + sx), Y = by - (oyi * G.L + sy);
  cplx mono, dip;
  sesm_green_pair(K, K.j, X, Y, &mono, &dip, lam == 0 ? 1 : 2);
  W[((int64_t)o * ns2 + s) * nb + b] = mono;
  W[((int64_t)o * ns2 + G.n_eq + s) * nb + b] = dip;
}

// Near-field blocks: rows = nodes of the cell, columns = the band of the cell's
// column; entry = operator entry for the source image in the band.  The
// Bloch phase e^{i alpha d shift} of a wrapped column is left out (applied to
// the density when the block is applied), so the blocks serve every
// incidence on the surface.
__global__ __launch_bounds__(256) void k_near_setup(KParams K, int n_x, const int* __restrict__ chunk_q,
                                                    const int* __restrict__ chunk_t0, int rows_per_chunk,
                                                    const int* __restrict__ occ_cell,
                                                    const int* __restrict__ occ_off, const int* __restrict__ perm,
                                                    const int* __restrict__ col_lo, const int* __restrict__ col_w,
                                                    const int64_t* __restrict__ near_off,
                                                    const double* __restrict__ x, const double* __restrict__ f,
                                                    const double* __restrict__ fp, const double* __restrict__ fpp,
                                                    const double* __restrict__ logw, cplx* __restrict__ blk) {
  // one workgroup per chunk of up to rows_per_chunk rows of one cell (the
  // rows of the forward map's near-field workgroups)
  const int q = chunk_q[blockIdx.x], t0 = chunk_t0[blockIdx.x];
  const int col = occ_cell[q] % n_x;
  const int off = occ_off[q], nq = occ_off[q + 1] - off;
  const int nr = min(rows_per_chunk, nq - t0);
  const int lo = col_lo[col], w = col_w[col];
  cplx* B = blk + near_off[q] + (int64_t)t0 * w;
  const int tot = nr * w;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = t0 + e / w, u = e % w;
    const int i = perm[off + t];
    int l = lo + u, shift = 0;
    if (l < 0) {
      l += K.N;
      shift = -1;
    } else if (l >= K.N) {
      l -= K.N;
      shift = 1;
    }
    cplx v;
    if (shift == 0 && l == i) {
      v = sesm_entry_diag(K, fp[i], fpp[i]);
    } else {
      const double X = x[i] - (x[l] + shift * K.d), Y = f[i] - f[l];
      v = sesm_entry_offdiag(K, logw, X, Y, fp[l], 1.0);
    }
    B[e] = v;
  }
}

// One launch for the three HBM streams of the forward map that need only mu
// (workgroups in this order):
//  * [0, n_occ): EqSources, dens[lam][cell][oo] = sum_t P[(off + t) nout + o] mu[perm[off + t]],
//    o = lam 2 n_eq + oo (eq. eq_source_point).  Lanes run over the outputs o
//    (rows of P are contiguous in o); G = LOC_NT / OW thread groups split the
//    cell's nodes and are summed through LDS.
//  * next n_mode_blocks: partial sums of the completion modes over chunks of
//    nodes, part[n][c] = sum_l e^{-i alpha_n x_l - i beta_n f_l} J_l dx mu_l (eq. M_eta).
//  * next n_chunks: the near field, y[perm[off + t]] = sum_u blk_q[t][u] mu[band_q(u)]
//    (intersecting part eq. final_correction_0, singular part eq. local_mat,
//    1/2 I) for up to NEAR_ROWS consecutive rows t of one cell q.
constexpr int LOC_NT = 256, NEAR_ROWS = 8;
struct LocalArgs {
  int N, n_occ, n_mode_blocks, n_chunks, n_eq, n_cells, n_x;
  const int* occ_cell;
  const int* occ_off;
  const int* perm;
  const void* P;     // EqSources operators: cplx, or cplxf in the mixed-precision map
  cplx* dens;
  const double* x;
  const double* f;
  const double* J;
  cplx* mode_part;
  const int* chunk_q;
  const int* chunk_t0;
  const int* col_lo;
  const int* col_w;
  const int64_t* near_off;
  const cplx* nearblk;
  int64_t dens_ld, mode_ld;  // batches: per-density strides of dens and mode_part
};

// The near-field work items: up to NEAR_ROWS consecutive rows of one
// occupied cell against the cyclic band of its near columns,
// y[perm[off + t]] = sum_u blk_q[t][u] mu[band_q(u)] (intersecting part
// eq. final_correction_0, singular part eq. local_mat, 1/2 I).  The items
// are independent HBM streams of stored blocks; besides the first launch of
// the forward map they fill the workgroups left idle by the latency-bound
// grid stages (merge + FFT, y convolution, inverse FFT), which carry ranges of
// them as extra workgroups after their own.
struct NearArgs {
  int N, n_x;
  const int* occ_cell;
  const int* occ_off;
  const int* perm;
  const int* chunk_q;
  const int* chunk_t0;
  const int* col_lo;
  const int* col_w;
  const int64_t* near_off;
  const cplx* nearblk;
};

// Item `it`, 256 threads (tid = 0..255 within their group): each thread runs
// over band columns tid, tid + 256, ... with all NEAR_ROWS row loads of a
// column in flight; a wrapped column's density carries the Bloch phase
// ph[s] = e^{i alpha_s d} of density s (or its conjugate); per density s and
// row r the wavefront sums go to
// rs[(s NEAR_ROWS + r) 4 + wave].  For several densities (NB >= 3) the rows are
// taken in two passes of half as many accumulators; each row's sum is formed
// in the same order either way, so every launch shape gives the same bits.
// WRAP: the item's band reaches past the period (only cells next to x = 0 or
// x = d); other items skip the per-column image test.
template <int NB, bool WRAP>
__device__ __forceinline__ void near_accum_band(const NearArgs& A, int q, int t0, int nr, int lo, int w, int tid,
                                                cplx* rs, const cplx* __restrict__ mu, int64_t ldm, const cplx* ph) {
  const int N = A.N;
  const cplx* blk = A.nearblk + A.near_off[q] + (int64_t)t0 * w;
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int RP = NB >= 3 ? NEAR_ROWS / 2 : NEAR_ROWS;
#pragma unroll
  for (int r0 = 0; r0 < NEAR_ROWS; r0 += RP) {
    if (r0 >= nr) break;  // uniform over the item's threads
    cplx acc[NB][RP];
#pragma unroll
    for (int s = 0; s < NB; ++s)
#pragma unroll
      for (int r = 0; r < RP; ++r) acc[s][r] = cplx{0.0, 0.0};
    for (int u = tid; u < w; u += 256) {
      int l = lo + u;
      cplx m[NB];
      if (WRAP) {
        const int wr = (l < 0) ? -1 : ((l >= N) ? 1 : 0);  // source image x_l + wr d
        l -= wr * N;
#pragma unroll
        for (int s = 0; s < NB; ++s) {
          m[s] = mu[s * ldm + l];
          if (wr != 0) m[s] = cmul_fixed(wr > 0 ? ph[s] : conj(ph[s]), m[s]);  // its density mu_l e^{i alpha d wr}
        }
      } else {
#pragma unroll
        for (int s = 0; s < NB; ++s) m[s] = mu[s * ldm + l];
      }
      cplx v[RP];
#pragma unroll
      for (int r = 0; r < RP; ++r) v[r] = load_stream(&blk[(int64_t)min(r0 + r, nr - 1) * w + u]);
#pragma unroll
      for (int s = 0; s < NB; ++s)
#pragma unroll
        for (int r = 0; r < RP; ++r) acc[s][r] = cmac(acc[s][r], v[r], m[s]);
    }
#pragma unroll
    for (int s = 0; s < NB; ++s)
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const cplx sm = wave_sum(acc[s][r]);
        if (lane == 0) rs[(s * NEAR_ROWS + r0 + r) * 4 + wv] = sm;
      }
  }
}

template <int NB>
__device__ __forceinline__ void near_accum(const NearArgs& A, int it, int tid, cplx* rs,
                                           const cplx* __restrict__ mu, int64_t ldm, const cplx* ph) {
  const int q = A.chunk_q[it], t0 = A.chunk_t0[it];
  const int off = A.occ_off[q], nq = A.occ_off[q + 1] - off;
  const int nr = min(NEAR_ROWS, nq - t0);
  const int col = A.occ_cell[q] % A.n_x;
  const int lo = A.col_lo[col], w = A.col_w[col];
  if (lo < 0 || lo + w > A.N)
    near_accum_band<NB, true>(A, q, t0, nr, lo, w, tid, rs, mu, ldm, ph);
  else
    near_accum_band<NB, false>(A, q, t0, nr, lo, w, tid, rs, mu, ldm, ph);
}

// After a workgroup barrier: thread tid < rows of item `it` adds the four
// wavefront sums of its row (fixed order) and stores it.
template <int NB>
__device__ __forceinline__ void near_store(const NearArgs& A, int it, int tid, const cplx* rs,
                                           cplx* __restrict__ y, int64_t ldy) {
  const int q = A.chunk_q[it], t0 = A.chunk_t0[it];
  const int off = A.occ_off[q], nq = A.occ_off[q + 1] - off;
  const int nr = min(NEAR_ROWS, nq - t0);
  if (tid < nr) {
    const int dst = A.perm[off + t0 + tid];
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      cplx sm = cplx{0.0, 0.0};
      for (int k = 0; k < 4; ++k) sm += rs[(s * NEAR_ROWS + tid) * 4 + k];
      y[s * ldy + dst] = sm;
    }
  }
}

// Near-field items [it0, it0 + GROUPS) (those below c1) for one density, by a
// workgroup of GROUPS x 256 threads: group g takes item it0 + g.
template <int GROUPS>
__device__ __forceinline__ void near_fill(const NearArgs& A, int it0, int c1, const cplx* __restrict__ mu,
                                          cplx* __restrict__ y, double alpha_d) {
  __shared__ cplx rs_fill[GROUPS * NEAR_ROWS * 4];
  const int g = threadIdx.x >> 8, tid = threadIdx.x & 255;
  const int it = it0 + g;
  cplx* rs = rs_fill + g * NEAR_ROWS * 4;
  const cplx ph = cexp_i(alpha_d);  // (formed as in the first launch: the same bits)
  if (it < c1) near_accum<1>(A, it, tid, rs, mu, 0, &ph);
  __syncthreads();
  if (it < c1) near_store<1>(A, it, tid, rs, y, 0);
}

// A range of near-field items carried by a launch: items [c0, c1) for the
// density mu, results into y.
struct NearFill {
  int c0, c1;
  const cplx* mu;
  cplx* y;
  double alpha_d;  // alpha d of the density's incidence
};


__host__ __device__ inline NearArgs near_args(const LocalArgs& L) {
  NearArgs A;
  A.N = L.N;
  A.n_x = L.n_x;
  A.occ_cell = L.occ_cell;
  A.occ_off = L.occ_off;
  A.perm = L.perm;
  A.chunk_q = L.chunk_q;
  A.chunk_t0 = L.chunk_t0;
  A.col_lo = L.col_lo;
  A.col_w = L.col_w;
  A.near_off = L.near_off;
  A.nearblk = L.nearblk;
  return A;
}

// The work of k_local_apply for NB densities at once: density r is
// mu + r ldm, its output y + r ldy, its cell densities dens + r dens_ld and its
// mode partial sums mode_part + r mode_ld.  Each P and near-field entry, and
// each mode factor, is loaded or formed once and used for all NB densities;
// every sum of density r is formed in the same order as for a single density,
// so a batch reproduces single forward maps bit for bit.
template <int NB, typename PT>
__device__ __forceinline__ void local_apply(const KParams& K, const LocalArgs& L, const cplx* __restrict__ mu,
                                            int64_t ldm, cplx* __restrict__ y, int64_t ldy,
                                            const IncParams* __restrict__ inc, int inc_step) {
  __shared__ cplx red[LOC_NT];
  __shared__ cplx mus[NB][LOC_NT];                 // EqSources: staged mu of the cell
  __shared__ cplx gsum[LOC_NT / 32][128];          // EqSources: per-group sums (one density at a time)
  int b = blockIdx.x;
  if (b < L.n_occ) {
    // EqSources of cell q: dens[o] = sum_t P[t][o] mu_t.  Lane l of each
    // 32-lane group holds outputs 4l..4l+3 (a 64-byte piece of a row of P);
    // the 8 groups take every 8th node, four nodes' loads in flight; the
    // cell's mu values are staged in LDS 256 at a time, and the groups'
    // sums are added in LDS in a fixed order.
    static_assert(LOC_NT == 256, "eight groups of 32 lanes");
    constexpr int OPL = 4, GL = 32, NG = LOC_NT / GL;
    constexpr int PU = NB >= 4 ? 1 : (NB >= 3 ? 2 : 4);  // nodes' loads in flight per group (registers: NB OPL sums)
    const int q = b;
    const int nout = 4 * L.n_eq;  // <= 128 = GL OPL
    const int g = threadIdx.x / GL, l = threadIdx.x % GL;
    const int cell = L.occ_cell[q];
    const int off = L.occ_off[q], nq = L.occ_off[q + 1] - off;
    cplx acc[NB][OPL];
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
      for (int j = 0; j < OPL; ++j) acc[r][j] = cplx{0.0, 0.0};
    const int oc = min(OPL * l, nout - OPL);  // lanes past the row repeat its last piece (not stored)
    for (int c0 = 0; c0 < nq; c0 += LOC_NT) {
      const int nc = min(LOC_NT, nq - c0);
      __syncthreads();
      if ((int)threadIdx.x < nc) {
        const int src = L.perm[off + c0 + threadIdx.x];
#pragma unroll
        for (int r = 0; r < NB; ++r) mus[r][threadIdx.x] = mu[r * ldm + src];
      }
      __syncthreads();
      const PT* pr = static_cast<const PT*>(L.P) + (int64_t)(off + c0) * nout + oc;
      int t = g;
      for (; t + (PU - 1) * NG < nc; t += PU * NG) {
        cplx v[PU][OPL];
#pragma unroll
        for (int u = 0; u < PU; ++u)
#pragma unroll
          for (int j = 0; j < OPL; ++j) v[u][j] = widen(pr[(int64_t)(t + u * NG) * nout + j]);
#pragma unroll
        for (int u = 0; u < PU; ++u)
#pragma unroll
          for (int r = 0; r < NB; ++r) {
            const cplx m = mus[r][t + u * NG];
#pragma unroll
            for (int j = 0; j < OPL; ++j) acc[r][j] = cmac(acc[r][j], v[u][j], m);
          }
      }
      for (; t < nc; t += NG) {
        cplx v[OPL];
#pragma unroll
        for (int j = 0; j < OPL; ++j) v[j] = widen(pr[(int64_t)t * nout + j]);
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          const cplx m = mus[r][t];
#pragma unroll
          for (int j = 0; j < OPL; ++j) acc[r][j] = cmac(acc[r][j], v[j], m);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      if (r > 0) __syncthreads();
#pragma unroll
      for (int j = 0; j < OPL; ++j) gsum[g][OPL * l + j] = acc[r][j];
      __syncthreads();
      if ((int)threadIdx.x < nout) {
        const int o = threadIdx.x;
        cplx sm = gsum[0][o];
        for (int gg = 1; gg < NG; ++gg) sm += gsum[gg][o];
        const int lam = o / (2 * L.n_eq), oo = o % (2 * L.n_eq);
        L.dens[r * L.dens_ld + ((int64_t)lam * L.n_cells + cell) * 2 * L.n_eq + oo] = sm;
      }
    }
    return;
  }
  b -= L.n_occ;
  if (b < L.n_mode_blocks) {
    // density r with the completion modes of its incidence inc[r inc_step]
    const int per = (K.N + NCH_MODES - 1) / NCH_MODES;
    const int lo = b * per, hi = min(K.N, lo + per);
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const IncParams& I = inc[r * inc_step];
      for (int t = 0; t < I.nU; ++t) {
        const double ua = I.Ua[t], ubr = I.Ubr[t], ubi = I.Ubi[t];
        cplx acc = cplx{0.0, 0.0};
        for (int l = lo + threadIdx.x; l < hi; l += LOC_NT) {
          const double mag = exp(ubi * L.f[l]) * L.J[l] * K.dx;
          const cplx e = mag * cexp_i(-(ua * L.x[l] + ubr * L.f[l]));
          acc = cmac(acc, e, mu[r * ldm + l]);
        }
        const cplx sm = block_sum<LOC_NT>(acc, red);
        if (threadIdx.x == 0) L.mode_part[r * L.mode_ld + (int64_t)t * NCH_MODES + b] = sm;
        __syncthreads();
      }
    }
    return;
  }
  b -= L.n_mode_blocks;
  // near-field work item b (the launch carries items [0, n_chunks))
  __shared__ cplx rs[NB * NEAR_ROWS * 4];  // near-field row sums per wavefront
  const NearArgs NA = near_args(L);
  cplx ph[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) ph[r] = cexp_i(inc[r * inc_step].alpha_d);
  near_accum<NB>(NA, b, threadIdx.x, rs, mu, ldm, ph);
  __syncthreads();
  near_store<NB>(NA, b, threadIdx.x, rs, y, ldy);
}

// PT: storage of the EqSources operators (cplx; cplxf in the mixed-precision map)
template <typename PT>
__global__ __launch_bounds__(LOC_NT) void k_local_apply(KParams K, LocalArgs L, const cplx* __restrict__ mu,
                                                        cplx* __restrict__ y, const IncParams* __restrict__ inc) {
  local_apply<1, PT>(K, L, mu, 0, y, 0, inc, 0);
}

// NB densities at once (strides ldm, ldy in elements).  At least four
// wavefronts per SIMD: for NB = 4 this caps the registers at 128 (a few values
// spill), one more workgroup per CU than the 133 the compiler would take, and
// the batched map of 8 densities runs 4.7% faster.
template <int NB, typename PT>
__global__ __launch_bounds__(LOC_NT, 4) void k_local_apply_batch(KParams K, LocalArgs L, const cplx* __restrict__ mu,
                                                              int64_t ldm, cplx* __restrict__ y, int64_t ldy,
                                                              const IncParams* __restrict__ inc, int inc_step) {
  local_apply<NB, PT>(K, L, mu, ldm, y, ldy, inc, inc_step);
}

// The near field of up to eight densities on the matrix cores (FP64 MFMA,
// 16 x 16 x 4): a workgroup takes 16 rows t of one occupied cell q and forms
// Y[t][s] = sum_u blk_q[t][u] mu_s[band_q(u)] for the densities s < nm as the
// real product [Re Y | Im Y] (16 x 16) = A (16 x 2w) B (2w x 16) with
//   A[t][2u + c] = (c = 0: Re, 1: Im) blk_q[t][u],
//   B[2u][s] = Re m_s(u), B[2u][8 + s] = Im m_s(u), B[2u + 1][s] = -Im m_s(u), B[2u + 1][8 + s] = Re m_s(u),
// m_s(u) the density of band column u (with its Bloch phase for a wrapped
// column).  Each of the four wavefronts takes a quarter of the columns
// (steps of two columns = one MFMA of K = 4) and the quarters are added in LDS
// in a fixed order.  Lane layouts of v_mfma_f64_16x16x4f64: A[l % 16][l / 16],
// B[l / 16][l % 16], D[4 r + l / 16][l % 16] in register r.
typedef double sesm_v4d __attribute__((ext_vector_type(4)));
constexpr int MF_COLS = 16;  // band columns per staged chunk and wavefront
__global__ __launch_bounds__(256) void k_near_mfma8(NearArgs NA, const int* __restrict__ tile_q,
                                                    const int* __restrict__ tile_t0, int nm,
                                                    const cplx* __restrict__ mu, int64_t ldm, cplx* __restrict__ y,
                                                    int64_t ldy, const IncParams* __restrict__ inc, int inc_step) {
  // per wavefront: the chunk's 16 rows x MF_COLS columns of the block (row
  // stride padded by one double against bank conflicts) and its densities
  constexpr int AS = 2 * MF_COLS + 1;
  __shared__ double As[4][16 * AS];
  __shared__ cplx Ms[4][MF_COLS * 8];
  __shared__ double red[4][4][64];
  const int q = tile_q[blockIdx.x], t0 = tile_t0[blockIdx.x];
  const int off = NA.occ_off[q], nq = NA.occ_off[q + 1] - off;
  const int nr = min(16, nq - t0);
  const int col = NA.occ_cell[q] % NA.n_x;
  const int lo = NA.col_lo[col], w = NA.col_w[col];
  const int N = NA.N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const cplx* blk = NA.nearblk + NA.near_off[q] + (int64_t)t0 * w;
  // this wavefront's columns [u_begin, u_end); every wavefront runs the same number of chunks
  const int quarter = ((w + 4 * MF_COLS - 1) / (4 * MF_COLS)) * MF_COLS;
  const int u_begin = min(w, wv * quarter), u_end = min(w, u_begin + quarter);
  // staging roles: block rows lane / 4 (clamped to the tile), columns 4 (lane % 4) .. + 3;
  // densities: member lane % 8, columns 2 (lane / 8) .. + 1
  const int sr = min(lane >> 2, nr - 1), sc = (lane & 3) * 4;
  const int ms = lane & 7, mc = (lane >> 3) * 2;
  cplx phs = cplx{1.0, 0.0};
  if (ms < nm) phs = cexp_i(inc[ms * inc_step].alpha_d);
  // MFMA roles
  const int kk = lane >> 4, i = lane & 15;
  const int s = i & 7, part = i >> 3, cb = kk & 1;
  double* Aw = As[wv];
  cplx* Mw = Ms[wv];
  sesm_v4d acc = {0.0, 0.0, 0.0, 0.0};
  // the next chunk's loads are issued before the current chunk's products
  cplx av[4], mv[2];
  auto load = [&](int ub) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int u = ub + sc + t;
      av[t] = u < u_end ? blk[(int64_t)sr * w + u] : cplx{0.0, 0.0};  // (plain loads: the non-temporal hint measured slower here)
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int u = ub + mc + t;
      cplx m = cplx{0.0, 0.0};
      if (u < u_end && ms < nm) {
        int l = lo + u;
        const int wr = (l < 0) ? -1 : ((l >= N) ? 1 : 0);
        l -= wr * N;
        m = mu[(int64_t)ms * ldm + l];
        if (wr != 0) m = cmul_fixed(wr > 0 ? phs : conj(phs), m);
      }
      mv[t] = m;
    }
  };
  load(u_begin);
  for (int c0 = 0; c0 < quarter; c0 += MF_COLS) {
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      Aw[(lane >> 2) * AS + 2 * (sc + t)] = av[t].re;
      Aw[(lane >> 2) * AS + 2 * (sc + t) + 1] = av[t].im;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) Mw[(mc + t) * 8 + ms] = mv[t];
    __syncthreads();
    if (c0 + MF_COLS < quarter) load(u_begin + c0 + MF_COLS);
#pragma unroll
    for (int st = 0; st < MF_COLS / 2; ++st) {
      const int ul = 2 * st + (kk >> 1);
      const double a = Aw[i * AS + 2 * ul + cb];
      const cplx m = Mw[ul * 8 + s];
      const double b = cb == 0 ? (part == 0 ? m.re : m.im) : (part == 0 ? -m.im : m.re);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv][r][lane] = acc[r];
  __syncthreads();
  // thread (r, l) of the sum: element D[4 r + l / 16][l % 16]
  const int r = threadIdx.x >> 6, l = threadIdx.x & 63;
  const double v = (red[0][r][l] + red[1][r][l]) + (red[2][r][l] + red[3][r][l]);
  const int row = 4 * r + (l >> 4), j = l & 15;
  if (row < nr && (j & 7) < nm) {
    const int dst = NA.perm[off + t0 + row];
    double* yd = reinterpret_cast<double*>(y + (int64_t)(j & 7) * ldy + dst);
    yd[j >> 3] = v;
  }
}

struct MergeArgs {
  int n_x, n_y, n_s, n_e, n_side, n_eq, n_cells;
  int nXH, nYH, nXV, nYV;
  double alpha_d;
};

// Local corrections (eq. small_convolution with the punctured kernel), by the
// workgroups from merge_blocks on of the y-convolution launch, for pairs
// p = (cell q, occupied cell rc of its near columns) at offset o:
// corr[p][b] = e^{i alpha d wr} sum_t W_o[t][b] dens_lambda(b)[rc][t].
struct CorrArgs {
  int n_groups, n_bdry, n_bH, n_eq, n_cells, merge_blocks;
  const int* grp_o;      // correction-matrix offset of each group
  const int* grp_start;  // its pairs: plist[grp_start .. grp_start + grp_n)
  const int* grp_n;
  const int* plist;      // pair indices, grouped by offset
  const int* grp_rc;     // source cell of each pair, in plist order
  const int* grp_wr;     // column wrap (-1, 0, 1) of each pair's source cell, in plist order
  const cplx* W;
  cplx* corr;
  int64_t bcorr, bdens;  // batched launches: corr and dens of batch member blockIdx.y are offset by these
  const IncParams* inc;  // incidence of member m: inc[m inc_step] (quasi-periodic phase of wrapped pairs)
  int inc_step;
};
constexpr int CORR_PPW = 3;              // pairs per wavefront
constexpr int CORR_PPB = 4 * CORR_PPW;   // pairs per correction workgroup (all share one matrix W_o)
constexpr int CORR_SB = 9;               // staged elements per thread and round (W_o up to 9 x 256 entries)

// dynamic LDS bytes of the correction workgroups: W_o and the pairs' densities
// (about 53 KB at n_s = 10: three workgroups per CU)
inline size_t corr_lds(int n_eq, int n_bdry) {
  return sizeof(cplx) * ((size_t)2 * n_eq * n_bdry + (size_t)CORR_PPB * 4 * n_eq);
}

// One workgroup per group of pairs with the same offset o: W_o and the pairs'
// source-cell densities are staged in LDS, and each W_o element serves several
// pairs at once (lambda of the boundary point: H rows use the horizontal set,
// V rows the vertical one).
__device__ inline void local_corr_group(const CorrArgs& C, const cplx* __restrict__ dens) {
  extern __shared__ cplx lds[];
  const int gi = blockIdx.x - C.merge_blocks;
  if (gi >= C.n_groups) return;  // block-uniform
  const int ns2 = 2 * C.n_eq, nb = C.n_bdry;
  const int o = C.grp_o[gi], p0 = C.grp_start[gi], np = C.grp_n[gi];
  cplx* Ws = lds;             // [ns2][nb]
  cplx* Ds = lds + ns2 * nb;  // [CORR_PPB][2 ns2]
  const cplx* Wo = C.W + (int64_t)o * ns2 * nb;
  const int tid = threadIdx.x, nW = ns2 * nb, nD = np * 2 * ns2;
  // staging in two memory latencies: the W_o loads and the source-cell indices
  // of this thread's density elements first, then the densities
  for (int e0 = tid; e0 < nW || e0 < nD; e0 += CORR_SB * 256) {
    cplx wv[CORR_SB], dv[CORR_SB];
    int rc[CORR_SB];
#pragma unroll
    for (int u = 0; u < CORR_SB; ++u) {
      wv[u] = Wo[min(e0 + u * 256, nW - 1)];
      rc[u] = C.grp_rc[p0 + min(e0 + u * 256, nD - 1) / (2 * ns2)];
    }
#pragma unroll
    for (int u = 0; u < CORR_SB; ++u) {
      const int t = min(e0 + u * 256, nD - 1) % (2 * ns2);
      dv[u] = dens[((int64_t)(t / ns2) * C.n_cells + rc[u]) * ns2 + t % ns2];
    }
#pragma unroll
    for (int u = 0; u < CORR_SB; ++u) {
      if (e0 + u * 256 < nW) Ws[e0 + u * 256] = wv[u];
      if (e0 + u * 256 < nD) Ds[e0 + u * 256] = dv[u];
    }
  }
  __syncthreads();
  // wavefront jg takes pairs CORR_PPW jg .. CORR_PPW jg + CORR_PPW - 1, lane b a
  // boundary point: independent sums share each W_o element
  const int b = tid & 63, jg = tid >> 6;
  if (b >= nb || CORR_PPW * jg >= np) return;
  const cplx* d = Ds + (size_t)(CORR_PPW * jg) * 2 * ns2 + (b < C.n_bH ? 0 : ns2);
  cplx acc[CORR_PPW];
#pragma unroll
  for (int j = 0; j < CORR_PPW; ++j) acc[j] = cplx{0.0, 0.0};
#pragma unroll 2
  for (int t = 0; t < ns2; ++t) {
    const cplx w = Ws[t * nb + b];
#pragma unroll
    for (int j = 0; j < CORR_PPW; ++j) acc[j] += w * d[j * 2 * ns2 + t];
  }
  const cplx php = cexp_i(C.inc[blockIdx.y * C.inc_step].alpha_d);
#pragma unroll
  for (int j = 0; j < CORR_PPW; ++j) {
    const int jj = CORR_PPW * jg + j;
    if (jj < np) {
      const int wr = C.grp_wr[p0 + jj];
      const cplx v = wr == 0 ? acc[j] : cmul_fixed(wr > 0 ? php : conj(php), acc[j]);
      C.corr[(int64_t)C.plist[p0 + jj] * nb + b] = v;
    }
  }
}

// Merged value of grid point (gy, gx) of one grid (eq. sum_eqsources): the
// densities of kind `kind` (0 = monopole xi, 1 = dipole zeta) of the up to six
// cell sides sharing the point (2 sides x 3 neighbours), with the
// quasi-periodic phase of a wrapped column and the twist exp(-i alpha x)
// (factor tw[gx]).  All candidate loads are issued before any is used.
__device__ inline cplx merge_point(const MergeArgs M, const cplx* __restrict__ dens, const cplx* __restrict__ tw,
                                   cplx php, bool onH, int kind, int gy, int gx) {
  const cplx* D = (onH ? dens : dens + (int64_t)M.n_cells * 2 * M.n_eq) + kind * M.n_eq;
  const cplx* src[6];
  int wr[6];
  bool ok[6];
#pragma unroll
  for (int side = 0; side < 2; ++side)
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
      const int id = side * 3 + d + 1;
      int row, c, pos, Wr = 0;
      if (onH) {  // bottom side of row gy, top side of row gy-1
        row = gy - side;
        c = gx / M.n_s + d;
        pos = gx - c * M.n_s;
      } else {    // left side of column gx, right side of column gx-1
        c = gx - side;
        row = (gy - M.n_e) / M.n_s + d;
        pos = gy - M.n_e - row * M.n_s;
      }
      ok[id] = row >= 0 && row < M.n_y && pos >= -M.n_e && pos <= M.n_s + M.n_e;
      if (c < 0) { c += M.n_x; Wr = -1; }
      else if (c >= M.n_x) { c -= M.n_x; Wr = 1; }
      wr[id] = Wr;
      src[id] = ok[id] ? D + (int64_t)(row * M.n_x + c) * 2 * M.n_eq + side * M.n_side + pos + M.n_e : D;
    }
  cplx va[6];
#pragma unroll
  for (int id = 0; id < 6; ++id) va[id] = src[id][0];
  const cplx twx = tw[gx];
  const cplx phm = conj(php);  // php = e^{i alpha d}
  cplx acc = cplx{0.0, 0.0};
#pragma unroll
  for (int id = 0; id < 6; ++id) {
    if (!ok[id]) continue;
    cplx v = va[id];
    if (wr[id] != 0) v = cmul_fixed(wr[id] > 0 ? php : phm, v);
    acc += v;
  }
  return acc * twx;
}

// Merge and forward x-FFT in one launch: the FFT workgroups of job jh (H grid,
// rows [kind][gy]) and then jv (V grid) gather their rows' merged values
// directly from the cell densities instead of reading a stored grid.
__global__ __launch_bounds__(1024) void k_merge_fft(MergeArgs M, const cplx* __restrict__ dens,
                                                    const cplx* __restrict__ twH, const cplx* __restrict__ twV,
                                                    FftJob jh, FftJob jv, NearArgs NA, NearFill F) {
  const int nfft = jh.nblocks + jv.nblocks;
  if ((int)blockIdx.x >= nfft) {  // near-field items, four per workgroup
    near_fill<4>(NA, F.c0 + 4 * ((int)blockIdx.x - nfft), F.c1, F.mu, F.y, F.alpha_d);
    return;
  }
  const bool onH = (int)blockIdx.x < jh.nblocks;
  const FftJob J = onH ? jh : jv;
  const int blk = onH ? blockIdx.x : blockIdx.x - jh.nblocks;
  const int nY = onH ? M.nYH : M.nYV;
  const cplx* tw = onH ? twH : twV;
  const cplx php = cexp_i(M.alpha_d);
  const MergeArgs Mv = M;
  sesm_fft_block(J, blk, -1, [=](int r, int i) { return merge_point(Mv, dens, tw, php, onH, r / nY, r % nY, i); });
}

// The same for several batch members: grid dimension y runs over them, member
// m reading dens + m fb.bin0 and writing the H grid at + m fb.bout0 and the V
// grid at + m fb.bout1.
__global__ __launch_bounds__(1024) void k_merge_fft_batch(MergeArgs M, const cplx* __restrict__ dens,
                                                          const cplx* __restrict__ twH, const cplx* __restrict__ twV,
                                                          FftJob jh, FftJob jv, FftBatch fb,
                                                          const IncParams* __restrict__ inc, int inc_step,
                                                          int64_t btw) {
  const bool onH = (int)blockIdx.x < jh.nblocks;
  FftJob J = onH ? jh : jv;
  const int64_t m = blockIdx.y;
  J.out += m * (onH ? fb.bout0 : fb.bout1);
  const cplx* db = dens + m * fb.bin0;
  const int blk = onH ? blockIdx.x : blockIdx.x - jh.nblocks;
  const int nY = onH ? M.nYH : M.nYV;
  const cplx* tw = (onH ? twH : twV) + m * btw;  // the member's twist e^{-i alpha_m x}
  const cplx php = cexp_i(inc[m * inc_step].alpha_d);
  const MergeArgs Mv = M;
  sesm_fft_block(J, blk, -1, [=](int r, int i) { return merge_point(Mv, db, tw, php, onH, r / nY, r % nY, i); });
}

// One grid of the y-direction convolution.
struct YConvJob {
  int nX, nY;
  const cplx* spec;  // kernel spectra [2][2nY-1][nX]
  const cplx* g;     // source spectra [2][nY][nX]
  cplx* out;         // [nY][nX]
  int64_t bg, bout;  // batched launches: g and out of batch member blockIdx.y are offset by these
  int64_t bspec;     // and its kernel spectra (incidence sets; 0 when the members share them)
};

// phi_hat[t][kx] = sum_t' spec0[t-t'+nY-1][kx] g0[t'][kx] + spec1[...] g1[t'][kx].
// Workgroups [0, hblocks) serve grid h, those up to C.merge_blocks grid v,
// and the rest compute the local corrections (above).  Short grids
// (nY <= 32) take 8 x-frequencies per workgroup (32 threads each); taller
// grids take one, with the sum over t' split in YC_SPLIT parts reduced in LDS.
// The columns (sources and kernel spectra) are gathered row-wise (coalesced
// over kx) into LDS first.
constexpr int YC_KPB = 8, YC_SPLIT = 4;
inline int yconv_kpb(int nY) { return nY <= 32 ? YC_KPB : 1; }
inline size_t yconv_lds(int nY) {
  const int per = 6 * nY - 2;
  return sizeof(cplx) * (nY <= 32 ? (size_t)YC_KPB * per : (size_t)per + YC_SPLIT * nY);
}
__global__ __launch_bounds__(256) void k_yconv(YConvJob h, YConvJob v, int hblocks, CorrArgs C,
                                               const cplx* __restrict__ dens, NearArgs NA, NearFill F) {
  extern __shared__ cplx col[];
  if ((int)blockIdx.x >= C.merge_blocks + C.n_groups) {  // near-field items, one per workgroup
    near_fill<1>(NA, F.c0 + (int)blockIdx.x - C.merge_blocks - C.n_groups, F.c1, F.mu, F.y, F.alpha_d);
    return;
  }
  if ((int)blockIdx.x >= C.merge_blocks) {  // the local corrections share the launch
    CorrArgs Cb = C;
    Cb.corr += (int64_t)blockIdx.y * C.bcorr;
    local_corr_group(Cb, dens + (int64_t)blockIdx.y * C.bdens);
    return;
  }
  const bool first = (int)blockIdx.x < hblocks;
  YConvJob J = first ? h : v;
  J.g += (int64_t)blockIdx.y * J.bg;
  J.out += (int64_t)blockIdx.y * J.bout;
  J.spec += (int64_t)blockIdx.y * J.bspec;
  const int b = first ? blockIdx.x : blockIdx.x - hblocks;
  const int nX = J.nX, nY = J.nY;
  const int nrow = 2 * nY - 1, per = 6 * nY - 2;
  const int kpb = nY <= 32 ? YC_KPB : 1;
  const int kx0 = b * kpb, nk = min(kpb, nX - kx0);
#pragma unroll 4
  for (int e = threadIdx.x; e < per * kpb; e += 256) {
    const int kl = e % kpb, r = e / kpb;
    if (kl < nk) {
      const int kx = kx0 + kl;
      col[kl * per + r] = r < 2 * nY ? J.g[(int64_t)r * nX + kx] : J.spec[(int64_t)(r - 2 * nY) * nX + kx];
    }
  }
  __syncthreads();
  if (kpb > 1) {
    const int kl = threadIdx.x >> 5, t = threadIdx.x & 31;
    if (kl < nk && t < nY) {
      const cplx* g0 = col + kl * per;
      const cplx* g1 = g0 + nY;
      const cplx* s0 = g0 + 2 * nY;
      const cplx* s1 = s0 + nrow;
      cplx a0 = cplx{0.0, 0.0}, a1 = cplx{0.0, 0.0};
      for (int tp = 0; tp < nY; ++tp) {
        const int r = t - tp + nY - 1;
        a0 += s0[r] * g0[tp];
        a1 += s1[r] * g1[tp];
      }
      J.out[(int64_t)t * nX + kx0 + kl] = a0 + a1;
    }
    return;
  }
  const cplx* g0 = col;
  const cplx* g1 = g0 + nY;
  const cplx* s0 = g0 + 2 * nY;
  const cplx* s1 = s0 + nrow;
  cplx* red = col + per;  // [YC_SPLIT][nY]
  const int TPT = 256 / YC_SPLIT, g = threadIdx.x / TPT, tt = threadIdx.x % TPT;
  const int chunk = (nY + YC_SPLIT - 1) / YC_SPLIT;
  const int lo = g * chunk, hi = min(nY, lo + chunk);
  for (int t = tt; t < nY; t += TPT) {
    cplx a0 = cplx{0.0, 0.0}, a1 = cplx{0.0, 0.0};
#pragma unroll 4
    for (int tp = lo; tp < hi; ++tp) {
      const int r = t - tp + nY - 1;
      a0 += s0[r] * g0[tp];
      a1 += s1[r] * g1[tp];
    }
    red[g * nY + t] = a0 + a1;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nY; t += 256) {
    cplx sm = red[t];
    for (int gg = 1; gg < YC_SPLIT; ++gg) sm += red[gg * nY + t];
    J.out[(int64_t)t * nX + kx0] = sm;
  }
}

// Inverse x-FFT of both grids (k_fft_rows) with near-field items as extra
// workgroups after the transform's (four per 1024-thread workgroup, one per
// 256-thread workgroup).
__global__ __launch_bounds__(1024) void k_fft_rows_near(FftJob j0, FftJob j1, int sign, NearArgs NA, NearFill F) {
  const int nfft = j0.nblocks + j1.nblocks;
  if ((int)blockIdx.x >= nfft) {
    if (blockDim.x == 1024)
      near_fill<4>(NA, F.c0 + 4 * ((int)blockIdx.x - nfft), F.c1, F.mu, F.y, F.alpha_d);
    else
      near_fill<1>(NA, F.c0 + (int)blockIdx.x - nfft, F.c1, F.mu, F.y, F.alpha_d);
    return;
  }
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

struct FarArgs {
  int N, n_x, n_y, n_s, n_e, n_side, n_eq, n_cells, n_bdry, n_bH, n_plw, nXH, nXV, ring, max_q;
  double L, x0, y0, k, alpha_d;
  // batched launches: per-member offsets of corr, phH, phV, mode_part and y
  int64_t bcorr, bphH, bphV, bmode, by;
  const int* cfc_q;   // work item -> occupied cell (null: one item per cell)
  const int* cfc_t0;  // work item -> its first node within the cell (max_q: nodes per item)
  cplx* bq_out;       // diagnostic: boundary values b^q of every occupied cell (null: not kept)
};

// One block per work item (up to max_q nodes of one occupied cell): the
// cell's boundary values of phi^all (H on horizontal sides incl. corners, V on
// vertical sides), minus the equivalent sources of the near columns (local
// corrections, from k_yconv), plane-wave weights, then the item's surface
// values plus the completion modes D_M (partial sums from k_local_apply).
// Dynamic LDS: the plane-wave factors ((U^H)^T, V^T, 1/sig), the item's nodes
// and their values.  Each phase keeps its global loads
// independent so that they are in flight together.
template <bool BATCHED>
__device__ __forceinline__ void cells_far_body(FarArgs A, KParams K, const int* __restrict__ occ_cell,
                                                   const int* __restrict__ occ_off, const int* __restrict__ perm,
                                                   const int* __restrict__ pair_off, const cplx* __restrict__ corr,
                                                   const cplx* __restrict__ phH, const cplx* __restrict__ phV,
                                                   const cplx* __restrict__ pplw, const double* __restrict__ dirs,
                                                   const double* __restrict__ x, const double* __restrict__ f,
                                                   const cplx* __restrict__ mode_part, cplx* __restrict__ y,
                                                   cplx* __restrict__ yfar, const IncParams* __restrict__ inc,
                                                   int inc_step) {
  extern __shared__ cplx dyn[];
  __shared__ cplx bv[64];
  __shared__ cplx wv_sh[64];
  __shared__ cplx msum[SESM_MAX_UETA];
  // the incidence of this member: Bloch phase of wrapped grid columns and completion modes
  const IncParams& I = inc[(BATCHED ? (int)blockIdx.y : 0) * inc_step];
  if (BATCHED) {  // batch member blockIdx.y
    const int64_t m = blockIdx.y;
    corr += m * A.bcorr;
    phH += m * A.bphH;
    phV += m * A.bphV;
    mode_part += m * A.bmode;
    y += m * A.by;
  }
  // work item: up to max_q consecutive nodes of occupied cell q (the cell's
  // boundary values and plane-wave weights are formed by each of its items)
  const int q = A.cfc_q ? A.cfc_q[blockIdx.x] : (int)blockIdx.x, t0c = A.cfc_q ? A.cfc_t0[blockIdx.x] : 0;
  const int cell = occ_cell[q];
  const int cx = cell % A.n_x, cy = cell / A.n_x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int off = occ_off[q] + t0c, nq = min(A.max_q, occ_off[q + 1] - off);
  const double ccx = A.x0 + (cx + 0.5) * A.L, ccy = A.y0 + (cy + 0.5) * A.L;
  const int npf = (A.n_bdry + A.n_plw + 1) * A.n_plw;  // plane-wave factors
  cplx* pf = dyn;
  cplx* ys = pf + npf;                                             // [max_q] surface values
  double* xs = reinterpret_cast<double*>(ys + A.max_q);            // [max_q] x, then [max_q] f
  int* node = reinterpret_cast<int*>(xs + 2 * A.max_q);            // [max_q] node index
  // phase 0: stage the plane-wave factors and the cell's nodes; completion-mode
  // sums (wave 1); boundary values of phi^all minus the local corrections of
  // the cell's pairs (threads b < n_bdry)
  stage_copy<10>(pf, pplw, npf, threadIdx.x, 256);
  for (int t = threadIdx.x; t < nq; t += 256) {
    const int i = perm[off + t];
    node[t] = i;
    xs[t] = x[i];
    xs[A.max_q + t] = f[i];
  }
  if (wv == 1) {
    for (int t = 0; t < I.nU; ++t) {
      cplx a = cplx{0.0, 0.0};
      for (int c = lane; c < NCH_MODES; c += 64) a += mode_part[(int64_t)t * NCH_MODES + c];
      a = wave_sum(a);
      if (lane == 0) msum[t] = a;
    }
  }
  if (threadIdx.x < A.n_bdry) {
    const int b = threadIdx.x;
    cplx val;
    if (b < A.n_bH) {
      const int iy = b / (A.n_s + 1), i = b % (A.n_s + 1);
      int gx = cx * A.n_s + i, Wr = 0;
      if (gx >= A.nXH) { gx -= A.nXH; Wr = 1; }
      val = phH[(int64_t)(cy + iy) * A.nXH + gx];
      if (Wr) val = cmul_fixed(cexp_i(I.alpha_d), val);
    } else {
      const int t = b - A.n_bH, ix = t / (A.n_s - 1), i = 1 + t % (A.n_s - 1);
      int gx = cx + ix, Wr = 0;
      if (gx >= A.nXV) { gx -= A.nXV; Wr = 1; }
      val = phV[(int64_t)(cy * A.n_s + i + A.n_e) * A.nXV + gx];
      if (Wr) val = cmul_fixed(cexp_i(I.alpha_d), val);
    }
    cplx cs = cplx{0.0, 0.0};
    const int p0 = pair_off[q], p1 = pair_off[q + 1];
#pragma unroll 8
    for (int p = p0; p < p1; ++p) cs += corr[(int64_t)p * A.n_bdry + b];
    bv[b] = val - cs;
    if (A.bq_out && t0c == 0) A.bq_out[(int64_t)q * A.n_bdry + b] = val - cs;
  }
  __syncthreads();
  // phase 3: plane-wave weights, the least squares of eq. plwave_QR through the
  // SVD of the plane-wave matrix, w = V diag(1/sig) U^H b: each product is
  // split over the four wavefronts (a quarter of the summation index each;
  // lane l holds output l) and the quarters are added in LDS in a fixed order;
  // V is stored transposed so that the lanes read V^T contiguously
  {
    __shared__ cplx p3[4][64];
    __shared__ cplx e_sh[64];
    const cplx* Vs = pf + A.n_bdry * A.n_plw;
    const cplx* isg = Vs + A.n_plw * A.n_plw;
    // U^H b: wavefront g sums its quarter of the boundary points
    {
      const int nb4 = (A.n_bdry + 3) / 4, b0 = wv * nb4, b1 = min(A.n_bdry, b0 + nb4);
      cplx acc = cplx{0.0, 0.0};
      if (lane < A.n_plw)
        for (int b = b0; b < b1; ++b) acc += pf[b * A.n_plw + lane] * bv[b];
      p3[wv][lane] = acc;
    }
    __syncthreads();
    if (threadIdx.x < A.n_plw) {
      const int l = threadIdx.x;
      e_sh[l] = isg[l].re * ((p3[0][l] + p3[1][l]) + (p3[2][l] + p3[3][l]));
    }
    __syncthreads();
    // w = V e: wavefront g sums its quarter of the directions
    {
      const int nj4 = (A.n_plw + 3) / 4, j0 = wv * nj4, j1 = min(A.n_plw, j0 + nj4);
      cplx acc = cplx{0.0, 0.0};
      if (lane < A.n_plw)
        for (int j = j0; j < j1; ++j) acc += Vs[j * A.n_plw + lane] * e_sh[j];
      p3[wv][lane] = acc;
    }
    __syncthreads();
    if (threadIdx.x < A.n_plw) {
      const int l = threadIdx.x;
      wv_sh[l] = (p3[0][l] + p3[1][l]) + (p3[2][l] + p3[3][l]);
    }
  }
  __syncthreads();
  // phase 4: surface values (eq. planewave), origin at the cell centre.  With
  // n_plw even, directions u and u + n_plw/2 are opposite, so one exponential
  // serves both (its conjugate).  Groups of UPL lanes take one node each.
  const bool pairs = (A.n_plw & 1) == 0;
  const int nd = pairs ? A.n_plw / 2 : A.n_plw;
  const int UPL = nd <= 16 ? 16 : (nd <= 32 ? 32 : 64);
  const int u = threadIdx.x & (UPL - 1), slot = threadIdx.x / UPL, nslot = 256 / UPL;
  double dxu = 0.0, dyu = 0.0;
  cplx wa = cplx{0.0, 0.0}, wb = cplx{0.0, 0.0};
  if (u < nd) {
    dxu = A.k * dirs[2 * u];
    dyu = A.k * dirs[2 * u + 1];
    wa = wv_sh[u];
    if (pairs) wb = wv_sh[u + nd];
  }
  for (int t0 = 0; t0 < nq; t0 += nslot) {  // uniform trip count (shuffles below)
    const int t = t0 + slot;
    cplx sv = cplx{0.0, 0.0};
    if (t < nq && u < nd) {
      const cplx e = cexp_i_reduced(dxu * (xs[t] - ccx) + dyu * (xs[A.max_q + t] - ccy));
      sv = wa * e + wb * conj(e);
    }
    if (UPL == 16) {
      sv.re = group_sum_d<16>(sv.re);
      sv.im = group_sum_d<16>(sv.im);
    } else if (UPL == 32) {
      sv.re = group_sum_d<32>(sv.re);
      sv.im = group_sum_d<32>(sv.im);
    } else {
      sv.re = group_sum_d<64>(sv.re);
      sv.im = group_sum_d<64>(sv.im);
    }
    if (t < nq && u == UPL - 1) ys[t] = sv;
  }
  __syncthreads();
  // phase 5: y_i += far value + completion modes sum_n e^{i alpha_n x_i + i beta_n f_i} s_n
  for (int t = threadIdx.x; t < nq; t += 256) {
    const int i = node[t];
    const cplx v = ys[t];
    cplx md = cplx{0.0, 0.0};
    for (int n = 0; n < I.nU; ++n) {
      const double mag = exp(-I.Ubi[n] * xs[A.max_q + t]);
      md += (mag * cexp_i(I.Ua[n] * xs[t] + I.Ubr[n] * xs[A.max_q + t])) * msum[n];
    }
    y[i] += v + md;
    if (yfar) yfar[i] = v;
  }
}

#define SESM_CELLS_FAR_PARAMS                                                                                       \
  FarArgs A, KParams K, const int *__restrict__ occ_cell, const int *__restrict__ occ_off,                         \
      const int *__restrict__ perm, const int *__restrict__ pair_off, const cplx *__restrict__ corr,              \
      const cplx *__restrict__ phH, const cplx *__restrict__ phV, const cplx *__restrict__ pplw,                 \
      const double *__restrict__ dirs, const double *__restrict__ x, const double *__restrict__ f,               \
      const cplx *__restrict__ mode_part, cplx *__restrict__ y, cplx *__restrict__ yfar,                           \
      const IncParams *__restrict__ inc, int inc_step
__global__ __launch_bounds__(256) void k_cells_far(SESM_CELLS_FAR_PARAMS) {
  cells_far_body<false>(A, K, occ_cell, occ_off, perm, pair_off, corr, phH, phV, pplw, dirs, x, f, mode_part, y, yfar,
                        inc, inc_step);
}
// grid dimension y: batch members (offsets in A)
__global__ __launch_bounds__(256) void k_cells_far_batch(SESM_CELLS_FAR_PARAMS) {
  cells_far_body<true>(A, K, occ_cell, occ_off, perm, pair_off, corr, phH, phV, pplw, dirs, x, f, mode_part, y, yfar,
                       inc, inc_step);
}
#undef SESM_CELLS_FAR_PARAMS

// dynamic LDS bytes of k_cells_far for work items of up to mq nodes
inline size_t cells_far_lds(const AccelOp* A, int mq_) {
  const size_t npf = (size_t)(A->n_bdry + A->n_plw + 1) * A->n_plw;
  const size_t mq = (size_t)mq_;
  return sizeof(cplx) * (npf + mq) + sizeof(double) * 2 * mq + sizeof(int) * mq;
}

template <typename T>
int upload(sesm_ctx* ctx, T** dst, const std::vector<T>& v) {
  int rc = sesm_alloc(ctx, (void**)dst, sizeof(T) * std::max<size_t>(v.size(), 1));
  if (rc) return rc;
  if (!v.empty()) {
    hipError_t e = hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return ctx->fail(SESM_EHIP, std::string("upload: ") + hipGetErrorString(e));
  }
  return SESM_OK;
}

CellGeo cell_geo(const AccelOp& A) {
  CellGeo G;
  G.n_s = A.n_s;
  G.n_e = A.n_e;
  G.n_side = A.n_side;
  G.n_eq = A.n_eq;
  G.n_coll = A.n_coll;
  G.L = A.L;
  G.delta = A.delta;
  return G;
}

// One launch of k_fft_rows for up to two jobs (j1 may be empty).
// Both jobs in one launch; members > 1 run the same jobs on further buffers
// (per-member offsets fb).
int fft_launch(sesm_ctx* ctx, hipStream_t st, const FftJob& j0, const FftJob& j1, int sign, int members = 1,
               FftBatch fb = FftBatch{}) {
  const int nb = j0.nblocks + j1.nblocks;
  if (nb == 0) return SESM_OK;
  const bool wide = (j0.nblocks && j0.A.n * j0.rpb >= 1000) || (j1.nblocks && j1.A.n * j1.rpb >= 1000);
  if (members > 1)
    hipLaunchKernelGGL(k_fft_rows_batch, dim3(nb, members), dim3(wide ? 1024 : 256), 0, st, j0, j1, sign, fb);
  else
    hipLaunchKernelGGL(k_fft_rows, dim3(nb), dim3(wide ? 1024 : 256), 0, st, j0, j1, sign);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}

constexpr double kHybridWindow = 8.0;
// The windowed lattice-sum tables (eq. Gq_limit with the Bloch phase of K.alpha)
// of both grids, twisted and transformed along x, into spec = [specH | specV].
int build_spectra(sesm_ctx* ctx, const KParams& K, cplx* spec) {
  AccelOp* A = ctx->acc;
  // the windowed rows of hybrid tables take a window kHybridWindow times wider
  // (their window error must stay far below that of a windowed table: next to
  // exact rows, a row's window error is a jump between rows that the
  // plane-wave fit of the cells amplifies)
  KParams Kw = K;
  if (A->hybrid) {
    Kw.A_len *= kHybridWindow;
    Kw.cA *= kHybridWindow;
  }
  const int pmax = (int)std::ceil(Kw.A_len / Kw.d) + 2;
  int rc;
  for (int lam = 0; lam < 2; ++lam) {
    const int nX = lam == 0 ? A->nXH : A->nXV, nY = lam == 0 ? A->nYH : A->nYV;
    const double hxs = lam == 0 ? A->delta : A->L, hys = lam == 0 ? A->L : A->delta;
    const int nrows = 2 * nY - 1;
    cplx* sp = spec + (lam == 0 ? 0 : (int64_t)2 * (2 * A->nYH - 1) * A->nXH);
    const AccelOp::HybridRows& H = A->hyb[lam];
    const int nmap = A->hybrid ? (int)H.spatial.size() : nrows;
    const int64_t ent = (int64_t)nmap * nX;
    if (ent > 0) {
      hipLaunchKernelGGL(k_lattice, dim3((unsigned)((ent + 3) / 4)), dim3(256), 0, ctx->stream, Kw, lam, nX, nY, hxs,
                         hys, pmax, A->hybrid ? H.d_spatial : nullptr, nmap, sp);
      SESM_LAUNCH_CHECK();
    }
    const FftJob J = sesm_fft_job(lam == 0 ? A->planH : A->planV, 2 * nrows, sp, sp, nullptr, nullptr, 1.0);
    if ((rc = fft_launch(ctx, ctx->stream, J, FftJob{}, -1))) return rc;
    if (A->hybrid && !H.spectral.empty()) {  // the spectral rows replace their (unfilled) transforms
      hipLaunchKernelGGL(k_spectral_rows, dim3((unsigned)H.spectral.size()), dim3(256), 0, ctx->stream, K, lam, nX,
                         nY, hys, H.d_spectral, H.d_nmax, sp);
      SESM_LAUNCH_CHECK();
    }
  }
  return SESM_OK;
}

// Which table rows the hybrid tables take from the spectral series (Sec. 3.2):
// at height Y the terms of mode n decay like e^{-|beta_n| delta}, delta =
// min_m |Y + m h| (eq. spectral_exp_estimate), so a row is spectral when delta > 0
// and the order nmax at which e^{-|beta_n| delta} < e^{-42} for every incidence
// (|alpha| < k) stays below kHybridMaxOrder; the rows close to a shifted pole
// row Y = -m h keep the windowed sums.
constexpr int kHybridMaxOrder = 40000;
int hybrid_rows(sesm_ctx* ctx, AccelOp* A) {
  const Problem& P = ctx->P;
  int rc;
  for (int lam = 0; lam < 2; ++lam) {
    AccelOp::HybridRows& H = A->hyb[lam];
    const int nY = lam == 0 ? A->nYH : A->nYV;
    const double hy = lam == 0 ? A->L : A->delta;
    H.spatial.clear();
    H.spectral.clear();
    H.nmax.clear();
    for (int row = 0; row < 2 * nY - 1; ++row) {
      const double Y = (row - (nY - 1)) * hy;
      double delta = 1e300;
      for (int m = 0; m <= P.j; ++m) delta = std::min(delta, std::fabs(Y + m * P.h));
      bool spectral = false;
      if (delta > 1e-9 * (P.h + hy)) {
        const double need = std::sqrt((42.0 / delta) * (42.0 / delta) + P.k * P.k) + P.k;
        const double nm = std::ceil(need * P.d / (2.0 * PI)) + 2.0;
        if (nm <= kHybridMaxOrder) {
          spectral = true;
          H.spectral.push_back(row);
          H.nmax.push_back((int)nm);
        }
      }
      if (!spectral) H.spatial.push_back(row);
    }
    if ((rc = upload(ctx, &H.d_spatial, H.spatial)) || (rc = upload(ctx, &H.d_spectral, H.spectral)) ||
        (rc = upload(ctx, &H.d_nmax, H.nmax)))
      return rc;
  }
  return SESM_OK;
}

// [e^{-i alpha x} on the H grid | on the V grid | e^{+i alpha x} on H | on V]
void twist_tables(const AccelOp* A, double alpha, std::vector<cplx>& tw) {
  tw.assign((size_t)A->tw_len, cplx{0.0, 0.0});
  for (int t = 0; t < A->nXH; ++t) {
    const double ph = alpha * t * A->delta;
    tw[t] = cplx{std::cos(ph), -std::sin(ph)};
    tw[A->nXH + A->nXV + t] = cplx{std::cos(ph), std::sin(ph)};
  }
  for (int t = 0; t < A->nXV; ++t) {
    const double ph = alpha * t * A->L;
    tw[A->nXH + t] = cplx{std::cos(ph), -std::sin(ph)};
    tw[2 * A->nXH + A->nXV + t] = cplx{std::cos(ph), std::sin(ph)};
  }
}

IncParams inc_record(const Problem& P) {
  IncParams I{};
  I.alpha = P.alpha;
  I.alpha_d = P.alpha * P.d;
  I.nU = P.nU;
  for (int t = 0; t < P.nU; ++t) {
    I.Ua[t] = P.Ua[t];
    I.Ubr[t] = P.Ubr[t];
    I.Ubi[t] = P.Ubi[t];
  }
  return I;
}

}  // namespace

void sesm_accel_free(sesm_ctx* ctx) {
  AccelOp* A = ctx->acc;
  delete A;  // device buffers are in ctx->owned
  ctx->acc = nullptr;
}

void sesm_accel_info(const sesm_ctx* ctx, sesm_surface_info* info) {
  const AccelOp* A = ctx->acc;
  if (!A) return;
  info->n_x = A->n_x;
  info->n_y = A->n_y;
  info->n_cells_occupied = A->n_occ;
  info->stencil_rows = A->n_y;
  info->L = A->L;
  info->y0 = A->y0;
  info->delta = A->delta;
  info->near_entries = A->near_entries;
  info->near_items[0] = A->near_c1;
  info->near_items[1] = A->near_c2 - A->near_c1;
  info->near_items[2] = A->near_c3 - A->near_c2;
  info->near_items[3] = A->n_chunks - A->near_c3;
  info->near_tuned_us = A->tuned_us;
  info->spectral_rows[0] = A->hybrid ? (int32_t)A->hyb[0].spectral.size() : 0;
  info->spectral_rows[1] = A->hybrid ? (int32_t)A->hyb[1].spectral.size() : 0;
}

static int choose_near_split(sesm_ctx* ctx);

int sesm_accel_setup(sesm_ctx* ctx) {
  const Problem& P = ctx->P;
  const sesm_params& prm = ctx->prm;
  const int N = P.N;
  AccelOp* A = new (std::nothrow) AccelOp();
  if (!A) return ctx->fail(SESM_ENOMEM, "host allocation failed");
  ctx->acc = A;
  A->n_s = prm.n_side ? prm.n_side : 10;
  A->n_e = prm.n_ext >= 0 ? (prm.n_ext ? prm.n_ext : 1) : 0;
  if (prm.n_ext < 0) A->n_e = 0;
  A->n_coll = prm.n_coll ? prm.n_coll : 6 * A->n_s;
  A->n_plw = prm.n_plw ? prm.n_plw : std::max(4, 4 * A->n_s - 8);
  A->ring = prm.near_ring ? prm.near_ring : 1;
  if (A->ring < 1 || A->ring > 3) return ctx->fail(SESM_EINVAL, "accelerator: near_ring must be 1, 2 or 3");
  if (A->n_s < 2 || A->n_s > 16 || A->n_e >= A->n_s || A->n_coll < 4 || A->n_coll > 256 || A->n_plw < 4 ||
      A->n_plw > 64)
    return ctx->fail(SESM_EINVAL, "accelerator: need 2 <= n_side <= 16, 0 <= n_ext < n_side, n_coll in [4,256], "
                                  "n_plw in [4,64]");
  A->n_x = smooth5_at_least(std::max(2 * A->ring + 1, (int)std::lround(P.d / prm.L_cell)));
  A->L = P.d / A->n_x;
  A->delta = A->L / A->n_s;
  if (!(P.a < A->L)) return ctx->fail(SESM_EINVAL, "accelerator: singular window a must be < L (Remark a_cond)");
  A->n_side = A->n_s + 1 + 2 * A->n_e;
  A->n_eq = 2 * A->n_side;
  if (A->n_side > 16)  // the EqSources lane layout holds 4 n_eq <= 128 outputs per cell
    return ctx->fail(SESM_EINVAL, "accelerator: n_side + 1 + 2 n_ext (equivalent sources per cell side) must be <= 16");
  A->n_bH = 2 * (A->n_s + 1);
  A->n_bdry = A->n_bH + 2 * (A->n_s - 1);
  if (A->n_bdry > 64) return ctx->fail(SESM_EINVAL, "accelerator: too many boundary points");
  // non-resonant cells (Remark non-resonant): -k^2 must not be a Dirichlet
  // eigenvalue of the L-square, (pi/L)^2 (m^2 + n^2) != k^2
  {
    const double kk = P.k * A->L / PI;
    const double t = kk * kk;
    for (int m = 1; m * m < t + 1; ++m)
      for (int n = 1; n * n + m * m < t + 1; ++n)
        if (std::fabs(m * m + n * n - t) < 1e-6 * t)
          return ctx->fail(SESM_ERESONANT, "accelerator: cell side L is a Dirichlet resonance of the square");
  }
  std::vector<double> hx(N), hf(N);
  SESM_HIP(hipMemcpyAsync(hx.data(), ctx->x, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipMemcpyAsync(hf.data(), ctx->f, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  A->x0 = -0.5 * P.dx;
  const double fmin = *std::min_element(hf.begin(), hf.end()), fmax = *std::max_element(hf.begin(), hf.end());
  A->n_y = (int)std::floor((fmax - fmin) / A->L) + 1;
  A->y0 = 0.5 * (fmin + fmax) - 0.5 * A->n_y * A->L;
  A->n_cells = A->n_x * A->n_y;
  A->nXH = A->n_x * A->n_s;
  A->nYH = A->n_y + 1;
  A->nXV = A->n_x;
  A->nYV = A->n_y * A->n_s + 1 + 2 * A->n_e;
  if (!sesm_fft_factor(A->nXH, &A->planH) || !sesm_fft_factor(A->nXV, &A->planV) || A->nXH > SESM_FFT_MAXN)
    return ctx->fail(SESM_EINVAL, "accelerator: periodic grid length must be 5-smooth and <= 2000");
  if (A->nYV > 400) return ctx->fail(SESM_EINVAL, "accelerator: surface too tall for the cell size (n_y n_s > 400)");
  // cells of the nodes, (a, b] convention
  std::vector<int> cellof(N), colof(N);
  for (int l = 0; l < N; ++l) {
    const int cxl = (int)std::ceil((hx[l] - A->x0) / A->L) - 1;
    const int cyl = (int)std::ceil((hf[l] - A->y0) / A->L) - 1;
    if (cxl < 0 || cxl >= A->n_x || cyl < 0 || cyl >= A->n_y)
      return ctx->fail(SESM_EINVAL, "accelerator: node outside the cell grid");
    colof[l] = cxl;
    cellof[l] = cyl * A->n_x + cxl;
  }
  std::vector<int> perm(N);
  for (int l = 0; l < N; ++l) perm[l] = l;
  std::stable_sort(perm.begin(), perm.end(), [&](int u, int v) { return cellof[u] < cellof[v]; });
  std::vector<int> occ_cell, occ_off;
  std::vector<unsigned char> occ_flag(A->n_cells, 0);
  for (int t = 0; t < N; ++t) {
    const int c = cellof[perm[t]];
    if (occ_cell.empty() || occ_cell.back() != c) {
      occ_cell.push_back(c);
      occ_off.push_back(t);
      occ_flag[c] = 1;
    }
  }
  occ_off.push_back(N);
  A->n_occ = (int)occ_cell.size();
  for (int q = 0; q < A->n_occ; ++q) A->max_q = std::max(A->max_q, occ_off[q + 1] - occ_off[q]);
  // column bands: nodes of columns c-ring..c+ring (cyclic), as a range [lo, lo + w)
  std::vector<int> first(A->n_x + 1, N);
  for (int l = N - 1; l >= 0; --l) first[colof[l]] = l;
  for (int c = A->n_x - 1; c >= 0; --c)
    if (first[c] > first[c + 1]) first[c] = first[c + 1];  // empty columns
  std::vector<int> col_lo(A->n_x), col_w(A->n_x);
  const int R = A->ring;
  for (int c = 0; c < A->n_x; ++c) {
    const int lo = c - R >= 0 ? first[c - R] : first[c - R + A->n_x] - N;
    const int hi = c + R + 1 <= A->n_x ? first[c + R + 1] : first[c + R + 1 - A->n_x] + N;
    col_lo[c] = lo;
    col_w[c] = hi - lo;
  }
  std::vector<int64_t> near_off(A->n_occ + 1, 0);
  for (int q = 0; q < A->n_occ; ++q)
    near_off[q + 1] = near_off[q] + (int64_t)(occ_off[q + 1] - occ_off[q]) * col_w[occ_cell[q] % A->n_x];
  A->near_entries = near_off[A->n_occ];
  // near-field work items: up to NEAR_ROWS rows of one cell
  std::vector<int> chunk_q, chunk_t0;
  for (int q = 0; q < A->n_occ; ++q)
    for (int t0 = 0; t0 < occ_off[q + 1] - occ_off[q]; t0 += NEAR_ROWS) {
      chunk_q.push_back(q);
      chunk_t0.push_back(t0);
    }
  A->n_chunks = (int)chunk_q.size();
  A->item_entries.assign(A->n_chunks + 1, 0);
  A->item_rows.assign(A->n_chunks + 1, 0);
  for (int it = 0; it < A->n_chunks; ++it) {
    const int q = chunk_q[it];
    const int rows = std::min(NEAR_ROWS, occ_off[q + 1] - occ_off[q] - chunk_t0[it]);
    A->item_rows[it + 1] = A->item_rows[it] + rows;
    A->item_entries[it + 1] = A->item_entries[it] + (int64_t)rows * col_w[occ_cell[q] % A->n_x];
  }
  // far-field work items: up to CF_NODES nodes of one cell
  std::vector<int> cfc_q, cfc_t0;
  for (int q = 0; q < A->n_occ; ++q)
    for (int t0 = 0; t0 < occ_off[q + 1] - occ_off[q]; t0 += CF_NODES) {
      cfc_q.push_back(q);
      cfc_t0.push_back(t0);
    }
  A->n_cfc = (int)cfc_q.size();
  for (int c = 0; c < A->n_x; ++c) A->max_w = std::max(A->max_w, col_w[c]);
  // tiles of the batched near field on the matrix cores: up to 16 rows of one cell
  std::vector<int> tile_q, tile_t0;
  A->batch_mfma = prm.batch_mfma == 1;
  if (A->batch_mfma)
    for (int q = 0; q < A->n_occ; ++q)
      for (int t0 = 0; t0 < occ_off[q + 1] - occ_off[q]; t0 += 16) {
        tile_q.push_back(q);
        tile_t0.push_back(t0);
      }
  A->n_tiles = (int)tile_q.size();
  int rc;
  if ((rc = upload(ctx, &A->occ_cell, occ_cell)) || (rc = upload(ctx, &A->occ_off, occ_off)) ||
      (rc = upload(ctx, &A->perm, perm)) || (rc = upload(ctx, &A->col_lo, col_lo)) ||
      (rc = upload(ctx, &A->col_w, col_w)) || (rc = upload(ctx, &A->near_off, near_off)) ||
      (rc = upload(ctx, &A->chunk_q, chunk_q)) || (rc = upload(ctx, &A->chunk_t0, chunk_t0)) ||
      (rc = upload(ctx, &A->cfc_q, cfc_q)) || (rc = upload(ctx, &A->cfc_t0, cfc_t0)) ||
      (rc = upload(ctx, &A->tile_q, tile_q)) || (rc = upload(ctx, &A->tile_t0, tile_t0)))
    return rc;
  // local-correction pairs: for every occupied cell, the occupied cells of its
  // 2 ring + 1 columns (all rows), with the correction-matrix offset and the
  // quasi-periodic phase of a wrapped column
  {
    const int nrowoff = 2 * A->n_y - 1;
    std::vector<int> pair_off(1, 0), pair_o, pair_rc, pair_wr;
    for (int q = 0; q < A->n_occ; ++q) {
      const int cx = occ_cell[q] % A->n_x, cy = occ_cell[q] / A->n_x;
      for (int dc = -R; dc <= R; ++dc)
        for (int ry = 0; ry < A->n_y; ++ry) {
          int col = cx + dc, Wr = 0;
          if (col < 0) { col += A->n_x; Wr = -1; }
          else if (col >= A->n_x) { col -= A->n_x; Wr = 1; }
          const int rcell = ry * A->n_x + col;
          if (!occ_flag[rcell]) continue;
          pair_o.push_back((dc + R) * nrowoff + (ry - cy + A->n_y - 1));
          pair_rc.push_back(rcell);
          pair_wr.push_back(Wr);
        }
      pair_off.push_back((int)pair_o.size());
    }
    A->n_pairs = (int)pair_o.size();
    // groups of at most CORR_PPB pairs sharing one offset (one correction matrix)
    std::vector<std::vector<int>> by_o((size_t)(2 * R + 1) * nrowoff);
    for (int p = 0; p < A->n_pairs; ++p) by_o[pair_o[p]].push_back(p);
    std::vector<int> grp_o, grp_start, grp_n, plist;
    for (int o = 0; o < (int)by_o.size(); ++o)
      for (size_t j0 = 0; j0 < by_o[o].size(); j0 += CORR_PPB) {
        grp_o.push_back(o);
        grp_start.push_back((int)plist.size());
        const int n = (int)std::min<size_t>(CORR_PPB, by_o[o].size() - j0);
        grp_n.push_back(n);
        for (int j = 0; j < n; ++j) plist.push_back(by_o[o][j0 + j]);
      }
    A->n_groups = (int)grp_o.size();
    std::vector<int> grp_rc(plist.size()), grp_wr(plist.size());
    for (size_t i = 0; i < plist.size(); ++i) {
      grp_rc[i] = pair_rc[plist[i]];
      grp_wr[i] = pair_wr[plist[i]];
    }
    if ((rc = upload(ctx, &A->pair_off, pair_off)) || (rc = upload(ctx, &A->grp_rc, grp_rc)) ||
        (rc = upload(ctx, &A->grp_wr, grp_wr)) || (rc = upload(ctx, &A->grp_o, grp_o)) ||
        (rc = upload(ctx, &A->grp_start, grp_start)) || (rc = upload(ctx, &A->grp_n, grp_n)) ||
        (rc = upload(ctx, &A->plist, plist)) ||
        (rc = sesm_alloc(ctx, (void**)&A->corr, sizeof(cplx) * (size_t)std::max(1, A->n_pairs) * A->n_bdry)))
      return rc;
    const size_t lds = std::max(std::max(yconv_lds(A->nYH), yconv_lds(A->nYV)), corr_lds(A->n_eq, A->n_bdry));
    if (lds > 140 * 1024) return ctx->fail(SESM_EINVAL, "accelerator: correction matrices exceed the LDS of a workgroup");
    if (lds > 64 * 1024)
      SESM_HIP(hipFuncSetAttribute((const void*)k_yconv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  const KParams K = ctx->kparams();
  const CellGeo G = cell_geo(*A);
  // --- equivalent-source least squares: A_eq (cell independent) on the
  // device, its QR on the host.  The surface-only tables are launched before
  // the factorisation so that the host work overlaps them.
  const int nrow = 4 * A->n_coll, ncol = 2 * A->n_eq;
  std::vector<C> hA((size_t)2 * nrow * ncol);
  {
    cplx* dA = nullptr;
    if ((rc = sesm_alloc(ctx, (void**)&dA, sizeof(cplx) * hA.size()))) return rc;
    for (int lam = 0; lam < 2; ++lam) {
      hipLaunchKernelGGL(k_aeq, dim3((nrow * A->n_eq + 255) / 256), dim3(256), 0, ctx->stream, K, G, lam,
                         dA + (size_t)lam * nrow * ncol);
      SESM_LAUNCH_CHECK();
    }
    SESM_HIP(hipMemcpyAsync(hA.data(), dA, sizeof(cplx) * hA.size(), hipMemcpyDeviceToHost, ctx->stream));
    SESM_HIP(hipStreamSynchronize(ctx->stream));
  }
  // --- global kernel tables and their spectra
  for (FftPlan* pl : {&A->planH, &A->planV}) {
    std::vector<cplx> tw(pl->n);
    for (int t = 0; t < pl->n; ++t) {
      const double ph = -2.0 * PI * t / pl->n;
      tw[t] = cplx{std::cos(ph), std::sin(ph)};
    }
    if ((rc = upload(ctx, &pl->tw, tw))) return rc;
  }
  A->spec_len = (int64_t)2 * (2 * A->nYH - 1) * A->nXH + (int64_t)2 * (2 * A->nYV - 1) * A->nXV;
  A->tw_len = (int64_t)2 * (A->nXH + A->nXV);
  if ((rc = sesm_alloc(ctx, (void**)&A->self_spec, sizeof(cplx) * (size_t)A->spec_len))) return rc;
  A->specH = A->self_spec;
  A->specV = A->self_spec + (int64_t)2 * (2 * A->nYH - 1) * A->nXH;
  A->hybrid = prm.table == 1;
  if (A->hybrid && (rc = hybrid_rows(ctx, A))) return rc;
  if ((rc = build_spectra(ctx, K, A->self_spec))) return rc;
  // --- local correction matrices
  A->n_off = (2 * A->ring + 1) * (2 * A->n_y - 1);
  {
    const size_t lds = cells_far_lds(A, A->max_q);  // whole cells (batched launches); items need less
    if (lds > 140 * 1024) return ctx->fail(SESM_EINVAL, "accelerator: plane-wave factors exceed the LDS of a workgroup");
    if (lds > 64 * 1024) {
      SESM_HIP(hipFuncSetAttribute((const void*)k_cells_far, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      SESM_HIP(
          hipFuncSetAttribute((const void*)k_cells_far_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
  }
  {
    const int64_t nW = (int64_t)A->n_off * A->n_bdry * ncol;
    if ((rc = sesm_alloc(ctx, (void**)&A->W, sizeof(cplx) * (size_t)nW))) return rc;
    const int64_t nth = (int64_t)A->n_off * A->n_bdry * A->n_eq;
    hipLaunchKernelGGL(k_wmat, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, ctx->stream, K, G, A->n_y, A->ring,
                       A->W);
    SESM_LAUNCH_CHECK();
  }
  // --- near-field blocks
  if ((rc = sesm_alloc(ctx, (void**)&A->nearblk, sizeof(cplx) * (size_t)std::max<int64_t>(A->near_entries, 1))))
    return rc;
  hipLaunchKernelGGL(k_near_setup, dim3(A->n_chunks), dim3(256), 0, ctx->stream, K, A->n_x, A->chunk_q,
                     A->chunk_t0, NEAR_ROWS, A->occ_cell, A->occ_off,
                     A->perm, A->col_lo, A->col_w, A->near_off, ctx->x, ctx->f, ctx->fp, ctx->fpp, ctx->logw,
                     A->nearblk);
  SESM_LAUNCH_CHECK();
  // --- QR of A_eq (both sets, one on a second host thread), while the device
  // builds the tables above
  {
    std::vector<C> Qh[2], Rm[2];
    bool ok[2] = {false, false};
    auto factor = [&](int lam) {
      std::vector<C> Al(hA.begin() + (size_t)lam * nrow * ncol, hA.begin() + (size_t)(lam + 1) * nrow * ncol);
      ok[lam] = ls_qr(nrow, ncol, std::move(Al), Qh[lam], Rm[lam]);
    };
    std::thread other;
    bool threaded = true;
    try {
      other = std::thread(factor, 1);
    } catch (...) {  // no second thread: factor both here
      threaded = false;
    }
    factor(0);
    if (threaded)
      other.join();
    else
      factor(1);
    if (!ok[0] || !ok[1]) return ctx->fail(SESM_EINVAL, "equivalent-source matrix is rank deficient");
    // per set: Q^H (ncol x nrow) and R (ncol x ncol), both stored column-major
    // (the P2E set-up's lanes run over the rows)
    std::vector<cplx> qr_all;
    for (int lam = 0; lam < 2; ++lam) {
      for (int c = 0; c < nrow; ++c)
        for (int j = 0; j < ncol; ++j) {
          const C v = Qh[lam][(size_t)j * nrow + c];
          qr_all.push_back(cplx{v.real(), v.imag()});
        }
      for (int r = 0; r < ncol; ++r)
        for (int u = 0; u < ncol; ++u) {
          const C v = Rm[lam][(size_t)u * ncol + r];
          qr_all.push_back(cplx{v.real(), v.imag()});
        }
    }
    if ((rc = upload(ctx, &A->pinv, qr_all))) return rc;
  }
  // --- P_q for every occupied cell
  if ((rc = sesm_alloc(ctx, (void**)&A->p2e, sizeof(cplx) * (size_t)4 * A->n_eq * N))) return rc;
  if (ncol > 64) return ctx->fail(SESM_EINVAL, "accelerator: at most 64 equivalent-source unknowns per set");
  hipLaunchKernelGGL(k_p2e_setup, dim3(A->n_chunks), dim3(256), sizeof(cplx) * 4 * nrow, ctx->stream, K, G,
                     A->x0, A->y0, A->n_x, A->chunk_q, A->chunk_t0, NEAR_ROWS, A->occ_cell, A->occ_off, A->perm, ctx->x, ctx->f, ctx->fp, A->pinv, A->p2e);
  SESM_LAUNCH_CHECK();
  if (prm.mixed) {  // FP32 copy of the EqSources operators for the mixed-precision map
    const int64_t n32 = (int64_t)4 * A->n_eq * N;
    if ((rc = sesm_alloc(ctx, (void**)&A->p2e32, sizeof(cplxf) * (size_t)n32))) return rc;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((n32 + 255) / 256)), dim3(256), 0, ctx->stream, n32, A->p2e, A->p2e32);
    SESM_LAUNCH_CHECK();
  }
  // --- twist factors of the global grids, and the incidence record
  {
    std::vector<cplx> tw;
    twist_tables(A, P.alpha, tw);
    if ((rc = upload(ctx, &A->self_tw, tw))) return rc;
    A->twxH = A->self_tw;
    A->twxV = A->self_tw + A->nXH;
    A->utwH = A->self_tw + A->nXH + A->nXV;
    A->utwV = A->self_tw + 2 * A->nXH + A->nXV;
    std::vector<IncParams> ip(1, inc_record(P));
    if ((rc = upload(ctx, &A->inc_self, ip))) return rc;
  }
  // --- plane waves: d_s = (sin 2 pi s / n_plw, cos 2 pi s / n_plw), s = 1..n_plw (eq. plwave_QR)
  {
    std::vector<double> dirs(2 * A->n_plw);
    for (int s = 0; s < A->n_plw; ++s) {
      const double t = 2.0 * PI * (s + 1) / A->n_plw;
      dirs[2 * s] = std::sin(t);
      dirs[2 * s + 1] = std::cos(t);
    }
    std::vector<C> E((size_t)A->n_bdry * A->n_plw);
    for (int b = 0; b < A->n_bdry; ++b) {
      double bx, by;
      G.bdry_point(b, &bx, &by);
      bx -= 0.5 * A->L;
      by -= 0.5 * A->L;
      for (int s = 0; s < A->n_plw; ++s)
        E[(size_t)b * A->n_plw + s] = std::exp(C(0.0, P.k * (dirs[2 * s] * bx + dirs[2 * s + 1] * by)));
    }
    if (A->n_bdry < A->n_plw) return ctx->fail(SESM_EINVAL, "accelerator: need n_plw <= boundary points (4 n_side)");
    // w = V diag(1/sig) U^H b: (U^H)^T, V^T and 1/sig for the cell kernel (the
    // three factors are applied one after the other, never multiplied out)
    std::vector<C> Uh, Vm;
    std::vector<double> sig;
    if (!ls_svd(A->n_bdry, A->n_plw, E, Uh, sig, Vm))
      return ctx->fail(SESM_EINVAL, "plane-wave matrix is rank deficient");
    std::vector<cplx> pv;
    for (int b = 0; b < A->n_bdry; ++b)
      for (int u = 0; u < A->n_plw; ++u) {
        const C v = Uh[(size_t)u * A->n_bdry + b];
        pv.push_back(cplx{v.real(), v.imag()});
      }
    for (int j = 0; j < A->n_plw; ++j)  // V transposed: lane l of the cell kernel reads V[l][j] contiguously in l
      for (int l = 0; l < A->n_plw; ++l) {
        const C v = Vm[(size_t)l * A->n_plw + j];
        pv.push_back(cplx{v.real(), v.imag()});
      }
    for (int u = 0; u < A->n_plw; ++u) pv.push_back(cplx{1.0 / sig[u], 0.0});
    if ((rc = upload(ctx, &A->pplw, pv)) || (rc = upload(ctx, &A->dirs, dirs))) return rc;
  }
  // --- work buffers
  const size_t nH = (size_t)A->nXH * A->nYH, nV = (size_t)A->nXV * A->nYV;
  if ((rc = sesm_alloc(ctx, (void**)&A->dens, sizeof(cplx) * (size_t)2 * A->n_cells * ncol)) ||
      (rc = sesm_alloc(ctx, (void**)&A->gH, sizeof(cplx) * 2 * nH)) ||
      (rc = sesm_alloc(ctx, (void**)&A->gV, sizeof(cplx) * 2 * nV)) ||
      (rc = sesm_alloc(ctx, (void**)&A->fH, sizeof(cplx) * 2 * nH)) ||
      (rc = sesm_alloc(ctx, (void**)&A->fV, sizeof(cplx) * 2 * nV)) ||
      (rc = sesm_alloc(ctx, (void**)&A->phH, sizeof(cplx) * nH)) ||
      (rc = sesm_alloc(ctx, (void**)&A->phV, sizeof(cplx) * nV)) ||
      (rc = sesm_alloc(ctx, (void**)&A->mode_part, sizeof(cplx) * SESM_MAX_UETA * NCH_MODES)) ||
      (rc = sesm_alloc(ctx, (void**)&A->yfar, sizeof(cplx) * (size_t)N)) ||
      (rc = sesm_alloc(ctx, (void**)&A->bq, sizeof(cplx) * (size_t)A->n_occ * A->n_bdry)))
    return rc;
  SESM_HIP(hipMemsetAsync(A->dens, 0, sizeof(cplx) * (size_t)2 * A->n_cells * ncol, ctx->stream));
  return choose_near_split(ctx);
}

// Algorithmic HBM bytes of one launch of each forward-map kernel (every
// input array read once, every output written once).
struct MatvecBytes {
  double local, merge, fftH0, fftH1, fftV0, fftV1, yconvH, yconvV, cells;
};

// near-field items [c0, c1): stored entries, and per row mu, y and the node
// index (16 + 16 + 4 bytes); per item the chunk tables (8 bytes)
static double near_bytes(const AccelOp* A, int c0, int c1) {
  if (c1 <= c0) return 0.0;
  const double ent = (double)(A->item_entries[c1] - A->item_entries[c0]);
  const double rows = (double)(A->item_rows[c1] - A->item_rows[c0]);
  return 16.0 * ent + rows * (2.0 * 16.0 + 4.0) + 8.0 * (c1 - c0);
}

// fill = true: the near-field items split over the launches as in a
// single-density forward map; false: all of them in the first launch
static MatvecBytes matvec_bytes(const sesm_ctx* ctx, bool fill) {
  const AccelOp* A = ctx->acc;
  const double N = ctx->P.N, c = sizeof(cplx);
  const double nout = 4.0 * A->n_eq, ns2 = 2.0 * A->n_eq;
  const double nH = (double)A->nXH * A->nYH, nV = (double)A->nXV * A->nYV;
  const double dens = c * 2.0 * A->n_cells * ns2;
  const int c1 = fill ? A->near_c1 : A->n_chunks, c2 = fill ? A->near_c2 : A->n_chunks,
            c3 = fill ? A->near_c3 : A->n_chunks;
  MatvecBytes B;
  // near field (its items in this launch), per-cell band start, width and
  // block offset (16 B); EqSources: operators, densities of the occupied
  // cells, cell tables (12 B); modes (when U^eta is not empty): x, f, J and
  // the partial sums
  B.local = near_bytes(A, 0, c1) + 16.0 * A->n_occ + c * nout * N + A->n_occ * (c * nout + 12.0) +
            (ctx->P.nU > 0 ? N * 24.0 + c * ctx->P.nU * NCH_MODES : 0.0);
  // merge + forward FFT: densities, twist factors and twiddles in, both
  // transformed grids (xi, zeta) out; near-field items carried along
  B.merge = dens + c * 2.0 * (A->nXH + A->nXV) + c * 2.0 * (nH + nV) + near_bytes(A, c1, c2);
  // inverse FFT: rows in + rows out, twiddle table, untwist factors
  B.fftH1 = c * (2.0 * A->nYH * A->nXH + 2.0 * A->nXH) + near_bytes(A, c3, A->n_chunks);
  B.fftV1 = c * (2.0 * A->nYV * A->nXV + 2.0 * A->nXV);
  B.fftH0 = B.fftV0 = 0.0;
  // spectra of both grids in, both kernel spectra, one output grid; local
  // corrections (correction matrices, densities, pair tables, corrections out)
  // counted with the H grid; near-field items carried along
  B.yconvH = c * (2.0 * nH + 2.0 * (2.0 * A->nYH - 1) * A->nXH + nH) + dens +
             c * (double)A->n_off * ns2 * A->n_bdry + A->n_pairs * (12.0 + c) + 12.0 * A->n_groups +
             c * (double)A->n_pairs * A->n_bdry + near_bytes(A, c2, c3);
  B.yconvV = c * (2.0 * nV + 2.0 * (2.0 * A->nYV - 1) * A->nXV + nV);
  // local corrections, phi grids, plane-wave SVD factors, directions, cell and pair
  // tables, node coordinates and index, y read and written, mode sums
  B.cells = c * (double)A->n_pairs * A->n_bdry + c * (nH + nV) +
            c * ((double)A->n_bdry * A->n_plw + (double)A->n_plw * A->n_plw + A->n_plw) + 16.0 * A->n_plw +
            16.0 * A->n_occ + N * (16.0 + 4.0 + 2.0 * c) + c * ctx->P.nU * NCH_MODES;
  return B;
}

static NearArgs near_args_host(const sesm_ctx* ctx) {
  const AccelOp* A = ctx->acc;
  NearArgs NA;
  NA.N = ctx->P.N;
  NA.n_x = A->n_x;
  NA.occ_cell = A->occ_cell;
  NA.occ_off = A->occ_off;
  NA.perm = A->perm;
  NA.chunk_q = A->chunk_q;
  NA.chunk_t0 = A->chunk_t0;
  NA.col_lo = A->col_lo;
  NA.col_w = A->col_w;
  NA.near_off = A->near_off;
  NA.nearblk = A->nearblk;
  return NA;
}

// Arguments of k_local_apply; without_far leaves only the near-field work items.
static LocalArgs local_args(const sesm_ctx* ctx, bool near_only) {
  const AccelOp* A = ctx->acc;
  LocalArgs L{};
  L.N = ctx->P.N;
  L.n_occ = near_only ? 0 : A->n_occ;
  L.n_mode_blocks = (near_only || ctx->P.nU == 0) ? 0 : NCH_MODES;
  L.n_chunks = A->n_chunks;
  L.n_eq = A->n_eq;
  L.n_cells = A->n_cells;
  L.n_x = A->n_x;
  L.occ_cell = A->occ_cell;
  L.occ_off = A->occ_off;
  L.perm = A->perm;
  L.P = A->p2e;
  L.dens = A->dens;
  L.x = ctx->x;
  L.f = ctx->f;
  L.J = ctx->J;
  L.mode_part = A->mode_part;
  L.chunk_q = A->chunk_q;
  L.chunk_t0 = A->chunk_t0;
  L.col_lo = A->col_lo;
  L.col_w = A->col_w;
  L.near_off = A->near_off;
  L.nearblk = A->nearblk;
  return L;
}

// Work buffers of the stages after the local launch, for nb densities at
// once: member m's buffers are the base pointers plus m times the strides.
struct FarBufs {
  int nb;
  const cplx *dens, *mode;
  cplx *fH, *fV, *gH, *gV, *phH, *phV, *corr, *y;
  int64_t bdens, bmode, bfH, bfV, bgH, bgV, bphH, bphV, bcorr, by;
  // incidence of member m: inc[m inc_step], spectra spec + m bspec, twist
  // factors tw + m btw (the tables' layout of AccelOp); alpha_d0 = alpha d of member 0
  const IncParams* inc;
  int inc_step;
  const cplx* spec;
  int64_t bspec;
  const cplx* tw;
  int64_t btw;
  double alpha_d0;
};

// the tables of the surface's own incidence, shared by every member
static void own_incidence(const sesm_ctx* ctx, FarBufs& Fb) {
  const AccelOp* A = ctx->acc;
  Fb.inc = A->inc_self;
  Fb.inc_step = 0;
  Fb.spec = A->self_spec;
  Fb.bspec = 0;
  Fb.tw = A->self_tw;
  Fb.btw = 0;
  Fb.alpha_d0 = ctx->P.alpha * ctx->P.d;
}

// The stages after the local launch: merge + forward FFT, y convolution +
// local corrections, inverse FFT, and the cell far field added to y, each one
// launch for all nb densities (grid dimension y = batch member).  dens and
// mode hold the densities' cell densities and mode partial sums; y holds
// their near fields.
// fill_mu (one density only): the near-field items of the split beyond the
// first launch are carried by the merge, y-convolution and inverse-FFT
// launches, for the density fill_mu, into Fb.y.
static int accel_far_stages(sesm_ctx* ctx, const FarBufs& Fb, bool keep_far, const MatvecBytes& B,
                            const cplx* fill_mu = nullptr) {
  AccelOp* A = ctx->acc;
  const Problem& P = ctx->P;
  const KParams K = ctx->kparams();
  hipStream_t st = ctx->stream;
  const int nb = Fb.nb;
  int rc;
  const NearArgs NA = near_args_host(ctx);
  NearFill fm{0, 0, nullptr, nullptr, 0.0}, fy = fm, ff = fm;
  if (fill_mu && nb == 1) {
    fm = NearFill{A->near_c1, A->near_c2, fill_mu, Fb.y, Fb.alpha_d0};
    fy = NearFill{A->near_c2, A->near_c3, fill_mu, Fb.y, Fb.alpha_d0};
    ff = NearFill{A->near_c3, A->n_chunks, fill_mu, Fb.y, Fb.alpha_d0};
  }
  MergeArgs M{A->n_x, A->n_y, A->n_s, A->n_e, A->n_side, A->n_eq, A->n_cells,
              A->nXH, A->nYH, A->nXV, A->nYV, Fb.alpha_d0};
  const cplx* twH = Fb.tw;                              // e^{-i alpha x}, H grid (member 0)
  const cplx* twV = Fb.tw + A->nXH;                     //                V grid
  const cplx* utH = Fb.tw + A->nXH + A->nXV;            // e^{+i alpha x}, H grid
  const cplx* utV = Fb.tw + 2 * A->nXH + A->nXV;        //                V grid
  const cplx* spH = Fb.spec;
  const cplx* spV = Fb.spec + (int64_t)2 * (2 * A->nYH - 1) * A->nXH;
  // merge + forward FFT along x of both grids (rows [kind][gy])
  SESM_KT_BEGIN(SESM_KT_MERGE, st);
  {
    const FftJob jh = sesm_fft_job(A->planH, 2 * A->nYH, nullptr, Fb.fH, nullptr, nullptr, 1.0);
    const FftJob jv = sesm_fft_job(A->planV, 2 * A->nYV, nullptr, Fb.fV, nullptr, nullptr, 1.0);
    if (nb > 1)
      hipLaunchKernelGGL(k_merge_fft_batch, dim3(jh.nblocks + jv.nblocks, nb), dim3(1024), 0, st, M, Fb.dens, twH,
                         twV, jh, jv, FftBatch{Fb.bdens, Fb.bfH, 0, Fb.bfV, 0, 0}, Fb.inc, Fb.inc_step, Fb.btw);
    else
      hipLaunchKernelGGL(k_merge_fft, dim3(jh.nblocks + jv.nblocks + (fm.c1 - fm.c0 + 3) / 4), dim3(1024), 0, st, M,
                         Fb.dens, twH, twV, jh, jv, NA, fm);
    SESM_LAUNCH_CHECK();
  }
  SESM_KT_END(SESM_KT_MERGE, st, nb * B.merge);
  // y convolution of both grids, with the local corrections in the same launch
  SESM_KT_BEGIN(SESM_KT_YCONV, st);
  {
    const YConvJob yh{A->nXH, A->nYH, spH, Fb.fH, Fb.gH, Fb.bfH, Fb.bgH, Fb.bspec};
    const YConvJob yv{A->nXV, A->nYV, spV, Fb.fV, Fb.gV, Fb.bfV, Fb.bgV, Fb.bspec};
    const int hb = (A->nXH + yconv_kpb(A->nYH) - 1) / yconv_kpb(A->nYH);
    const int vb = (A->nXV + yconv_kpb(A->nYV) - 1) / yconv_kpb(A->nYV);
    const CorrArgs CA{A->n_groups, A->n_bdry, A->n_bH,   A->n_eq,   A->n_cells, hb + vb,  A->grp_o,
                      A->grp_start, A->grp_n, A->plist, A->grp_rc, A->grp_wr, A->W,      Fb.corr,
                      Fb.bcorr,     Fb.bdens,  Fb.inc,   Fb.inc_step};
    const size_t lds = std::max(std::max(yconv_lds(A->nYH), yconv_lds(A->nYV)), corr_lds(A->n_eq, A->n_bdry));
    hipLaunchKernelGGL(k_yconv, dim3(hb + vb + A->n_groups + (fy.c1 - fy.c0), nb), dim3(256), lds, st, yh, yv, hb,
                       CA, Fb.dens, NA, fy);
    SESM_LAUNCH_CHECK();
  }
  SESM_KT_END(SESM_KT_YCONV, st, nb * (B.yconvH + B.yconvV));
  SESM_KT_BEGIN(SESM_KT_FFT, st);
  {
    const FftJob jh = sesm_fft_job(A->planH, A->nYH, Fb.gH, Fb.phH, nullptr, utH, 1.0 / A->nXH);
    const FftJob jv = sesm_fft_job(A->planV, A->nYV, Fb.gV, Fb.phV, nullptr, utV, 1.0 / A->nXV);
    if (ff.c1 > ff.c0) {  // one density with near-field items: the carrying variant
      const bool wide = (jh.nblocks && jh.A.n * jh.rpb >= 1000) || (jv.nblocks && jv.A.n * jv.rpb >= 1000);
      const int per = wide ? 4 : 1, nfill = (ff.c1 - ff.c0 + per - 1) / per;
      hipLaunchKernelGGL(k_fft_rows_near, dim3(jh.nblocks + jv.nblocks + nfill), dim3(wide ? 1024 : 256), 0, st, jh,
                         jv, +1, NA, ff);
      SESM_LAUNCH_CHECK();
    } else if ((rc = fft_launch(ctx, st, jh, jv, +1, nb, FftBatch{Fb.bgH, Fb.bphH, Fb.bgV, Fb.bphV, Fb.btw, Fb.btw}))) {
      return rc;
    }
  }
  SESM_KT_END(SESM_KT_FFT, st, nb * (B.fftH1 + B.fftV1));
  // one density: work items of up to CF_NODES nodes (the fullest cells no
  // longer set the length of the launch); several: one workgroup per cell and
  // member (the members already fill the chip)
  const bool items = nb == 1;
  const int mq = items ? std::min(A->max_q, CF_NODES) : A->max_q;
  FarArgs F{P.N,    A->n_x,   A->n_y,   A->n_s,    A->n_e, A->n_side, A->n_eq, A->n_cells, A->n_bdry, A->n_bH,
            A->n_plw, A->nXH, A->nXV,   A->ring,   mq,     A->L,   A->x0,     A->y0,   P.k,        Fb.alpha_d0,
            Fb.bcorr, Fb.bphH, Fb.bphV, Fb.bmode, Fb.by, items ? A->cfc_q : nullptr, items ? A->cfc_t0 : nullptr,
            keep_far ? A->bq : nullptr};
  SESM_KT_BEGIN(SESM_KT_CELLS, st);
  hipLaunchKernelGGL(nb > 1 ? k_cells_far_batch : k_cells_far, dim3(items ? A->n_cfc : A->n_occ, nb), dim3(256),
                     cells_far_lds(A, mq), st, F, K, A->occ_cell,
                     A->occ_off, A->perm, A->pair_off, Fb.corr, Fb.phH, Fb.phV, A->pplw, A->dirs, ctx->x, ctx->f,
                     Fb.mode, Fb.y, keep_far ? A->yfar : nullptr, Fb.inc, nb > 1 ? Fb.inc_step : 0);
  SESM_LAUNCH_CHECK();
  SESM_KT_END(SESM_KT_CELLS, st, nb * B.cells);
  return SESM_OK;
}

// mixed: the mixed-precision map (EqSources operators in FP32, products in FP64)
static int accel_matvec_impl(sesm_ctx* ctx, const cplx* mu, cplx* y, bool keep_far, bool mixed = false) {
  AccelOp* A = ctx->acc;
  const KParams K = ctx->kparams();
  hipStream_t st = ctx->stream;
  const MatvecBytes B = ctx->kt_mask ? matvec_bytes(ctx, true) : MatvecBytes{};
  LocalArgs L = local_args(ctx, false);
  L.n_chunks = A->near_c1;  // the other near-field items ride on the grid stages
  if (mixed && !A->p2e32) return ctx->fail(SESM_EINVAL, "mixed-precision map: surface set up without sesm_params.mixed");
  SESM_KT_BEGIN(SESM_KT_LOCAL, st);
  if (mixed) {
    L.P = A->p2e32;
    hipLaunchKernelGGL(k_local_apply<cplxf>, dim3(L.n_occ + L.n_mode_blocks + L.n_chunks), dim3(LOC_NT), 0, st, K, L,
                       mu, y, A->inc_self);
  } else {
    hipLaunchKernelGGL(k_local_apply<cplx>, dim3(L.n_occ + L.n_mode_blocks + L.n_chunks), dim3(LOC_NT), 0, st, K, L,
                       mu, y, A->inc_self);
  }
  SESM_LAUNCH_CHECK();
  SESM_KT_END(SESM_KT_LOCAL, st, B.local);
  FarBufs Fb{};
  Fb.nb = 1;
  Fb.dens = A->dens;
  Fb.mode = A->mode_part;
  Fb.fH = A->fH;
  Fb.fV = A->fV;
  Fb.gH = A->gH;
  Fb.gV = A->gV;
  Fb.phH = A->phH;
  Fb.phV = A->phV;
  Fb.corr = A->corr;
  Fb.y = y;
  own_incidence(ctx, Fb);
  return accel_far_stages(ctx, Fb, keep_far, B, mu);
}

template <int NB>
static void launch_local_batch(hipStream_t st, const KParams& K, const LocalArgs& L, const cplx* mu, int64_t ldm,
                               cplx* y, int64_t ldy, const IncParams* inc, int inc_step, bool mixed) {
  const dim3 grid(L.n_occ + L.n_mode_blocks + L.n_chunks);
  if (mixed)
    hipLaunchKernelGGL((k_local_apply_batch<NB, cplxf>), grid, dim3(LOC_NT), 0, st, K, L, mu, ldm, y, ldy, inc,
                       inc_step);
  else
    hipLaunchKernelGGL((k_local_apply_batch<NB, cplx>), grid, dim3(LOC_NT), 0, st, K, L, mu, ldm, y, ldy, inc,
                       inc_step);
}

// Forward maps of nrhs densities (column r at mu + r ldm, output at y + r ldy)
// in groups of up to kBatchMax densities: one local launch per group reads the
// near-field blocks and P once for the group, and each later stage is one
// launch for the group.
int sesm_accel_matvec_batch(sesm_ctx* ctx, int nrhs, const cplx* mu, int64_t ldm, cplx* y, int64_t ldy, int inc0,
                            bool mixed) {
  AccelOp* A = ctx->acc;
  if (mixed && !A->p2e32) return ctx->fail(SESM_EINVAL, "mixed-precision map: surface set up without sesm_params.mixed");
  if (inc0 >= 0 && (inc0 + nrhs > A->n_inc || !A->inc_set))
    return ctx->fail(SESM_EINVAL, "incidence index beyond the incidence set");
  const KParams K = ctx->kparams();
  hipStream_t st = ctx->stream;
  const size_t nH = (size_t)A->nXH * A->nYH, nV = (size_t)A->nXV * A->nYV;
  const size_t dens_n = (size_t)2 * A->n_cells * 2 * A->n_eq, mode_n = (size_t)SESM_MAX_UETA * NCH_MODES;
  const size_t corr_n = (size_t)std::max(1, A->n_pairs) * A->n_bdry;
  // per member: dens, mode, fH, fV, gH, gV, phH, phV, corr
  const size_t per[9] = {dens_n, mode_n, 2 * nH, 2 * nV, 2 * nH, 2 * nV, nH, nV, corr_n};
  int rc;
  if (!A->batch_ws) {
    size_t tot = 0;
    for (size_t v : per) tot += v;
    if ((rc = sesm_alloc(ctx, (void**)&A->batch_ws, sizeof(cplx) * tot * kBatchMax))) return rc;
    // cells without nodes are never written: their densities stay zero
    SESM_HIP(hipMemsetAsync(A->batch_ws, 0, sizeof(cplx) * dens_n * kBatchMax, st));
  }
  cplx* base[9];
  {
    cplx* p = A->batch_ws;
    for (int i = 0; i < 9; ++i) {
      base[i] = p;
      p += per[i] * kBatchMax;
    }
  }
  const MatvecBytes B = ctx->kt_mask ? matvec_bytes(ctx, false) : MatvecBytes{};  // per density (later stages)
  LocalArgs L = local_args(ctx, false);
  if (mixed) L.P = A->p2e32;
  L.dens = base[0];
  L.mode_part = base[1];
  L.dens_ld = (int64_t)dens_n;
  L.mode_ld = (int64_t)mode_n;
  FarBufs Fb{};
  Fb.dens = base[0];
  Fb.mode = base[1];
  Fb.fH = base[2];
  Fb.fV = base[3];
  Fb.gH = base[4];
  Fb.gV = base[5];
  Fb.phH = base[6];
  Fb.phV = base[7];
  Fb.corr = base[8];
  Fb.bdens = (int64_t)per[0];
  Fb.bmode = (int64_t)per[1];
  Fb.bfH = (int64_t)per[2];
  Fb.bfV = (int64_t)per[3];
  Fb.bgH = (int64_t)per[4];
  Fb.bgV = (int64_t)per[5];
  Fb.bphH = (int64_t)per[6];
  Fb.bphV = (int64_t)per[7];
  Fb.bcorr = (int64_t)per[8];
  Fb.by = ldy;
  const bool mfma = A->batch_mfma && A->n_tiles > 0;
  if (mfma) {
    // the near field of groups of up to eight densities on the matrix cores;
    // the local launches below then carry the EqSources and mode sums only
    L.n_chunks = 0;
    const NearArgs NA = near_args(L);
    for (int r0 = 0; r0 < nrhs; r0 += 8) {
      const int nm = std::min(8, nrhs - r0);
      const IncParams* ip = inc0 < 0 ? A->inc_self : A->inc_set + inc0 + r0;
      hipLaunchKernelGGL(k_near_mfma8, dim3(A->n_tiles), dim3(256), 0, st, NA, A->tile_q, A->tile_t0, nm,
                         mu + r0 * ldm, ldm, y + r0 * ldy, ldy, ip, inc0 < 0 ? 0 : 1);
      SESM_LAUNCH_CHECK();
    }
  }
  for (int r0 = 0; r0 < nrhs; r0 += kBatchMax) {
    const int nb = std::min(kBatchMax, nrhs - r0);
    const cplx* m0 = mu + r0 * ldm;
    cplx* y0 = y + r0 * ldy;
    if (inc0 < 0) {  // one operator for all: the surface's own incidence
      own_incidence(ctx, Fb);
    } else {         // densities r0.. with members inc0 + r0.. of the incidence set
      const int i0 = inc0 + r0;
      Fb.inc = A->inc_set + i0;
      Fb.inc_step = 1;
      Fb.spec = A->inc_spec + (int64_t)i0 * A->spec_len;
      Fb.bspec = A->spec_len;
      Fb.tw = A->inc_tw + (int64_t)i0 * A->tw_len;
      Fb.btw = A->tw_len;
      Fb.alpha_d0 = A->inc_prob[i0].alpha * ctx->P.d;
      bool modes = false;
      for (int r = 0; r < nb; ++r) modes = modes || A->inc_prob[i0 + r].nU > 0;
      L.n_mode_blocks = modes ? NCH_MODES : 0;
    }
    switch (nb) {
      case 1: launch_local_batch<1>(st, K, L, m0, ldm, y0, ldy, Fb.inc, Fb.inc_step, mixed); break;
      case 2: launch_local_batch<2>(st, K, L, m0, ldm, y0, ldy, Fb.inc, Fb.inc_step, mixed); break;
      case 3: launch_local_batch<3>(st, K, L, m0, ldm, y0, ldy, Fb.inc, Fb.inc_step, mixed); break;
      default: launch_local_batch<4>(st, K, L, m0, ldm, y0, ldy, Fb.inc, Fb.inc_step, mixed); break;
    }
    SESM_LAUNCH_CHECK();
    Fb.nb = nb;
    Fb.y = y0;
    if ((rc = accel_far_stages(ctx, Fb, false, B))) return rc;
  }
  return SESM_OK;
}

int sesm_accel_matvec(sesm_ctx* ctx, const cplx* mu, cplx* y, bool mixed) {
  return accel_matvec_impl(ctx, mu, y, false, mixed);
}

// give a block allocated with sesm_alloc back to the context's pool
static void accel_release(sesm_ctx* ctx, void* p) {
  if (!p) return;
  for (size_t t = 0; t < ctx->owned.size(); ++t)
    if (ctx->owned[t].first == p) {
      ctx->bytes -= (int64_t)ctx->owned[t].second;
      sesm_pool_put(ctx, p, ctx->owned[t].second);
      ctx->owned.erase(ctx->owned.begin() + t);
      return;
    }
}

// The incidence set: for every alpha_r, the problem's incidence-dependent
// scalars (completion set U^eta of eq. M_eta, propagating orders), the
// kernel spectra of the windowed lattice sums with the Bloch phase
// e^{-i alpha_r d p} (eq. Gq_limit), the twist factors and the device record.
// Everything else of the operator (near-field blocks, EqSources operators,
// local-correction matrices, plane-wave factors) does not depend on alpha
// and is shared.
int sesm_accel_set_incidences(sesm_ctx* ctx, int n, const double* alpha) {
  AccelOp* A = ctx->acc;
  const Problem& P = ctx->P;
  for (int r = 0; r < n; ++r)
    if (!std::isfinite(alpha[r]) || !(std::fabs(alpha[r]) < P.k))
      return ctx->fail(SESM_EINVAL, "incidence set: need |alpha| < k for every member");
  std::vector<Problem> probs(n, P);
  std::vector<IncParams> recs(n);
  for (int r = 0; r < n; ++r) {
    if (!sesm_problem_alpha(probs[r], alpha[r], P.eta))
      return ctx->fail(SESM_EINVAL, "incidence set: more than 64 completion modes; lower eta");
    recs[r] = inc_record(probs[r]);
  }
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  accel_release(ctx, A->inc_set);
  accel_release(ctx, A->inc_spec);
  accel_release(ctx, A->inc_tw);
  A->inc_set = nullptr;
  A->inc_spec = A->inc_tw = nullptr;
  A->n_inc = 0;
  A->inc_prob.clear();
  if (n == 0) return SESM_OK;
  int rc;
  if ((rc = upload(ctx, &A->inc_set, recs))) return rc;
  if ((rc = sesm_alloc(ctx, (void**)&A->inc_spec, sizeof(cplx) * (size_t)n * A->spec_len))) return rc;
  std::vector<cplx> tw_all((size_t)n * A->tw_len), tw;
  for (int r = 0; r < n; ++r) {
    KParams K = ctx->kparams();
    K.alpha = alpha[r];
    if ((rc = build_spectra(ctx, K, A->inc_spec + (int64_t)r * A->spec_len))) return rc;
    twist_tables(A, alpha[r], tw);
    std::copy(tw.begin(), tw.end(), tw_all.begin() + (int64_t)r * A->tw_len);
  }
  if ((rc = upload(ctx, &A->inc_tw, tw_all))) return rc;
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  A->inc_prob = std::move(probs);
  A->n_inc = n;
  return SESM_OK;
}

int sesm_accel_n_incidences(const sesm_ctx* ctx) { return ctx->acc ? ctx->acc->n_inc : 0; }

const Problem* sesm_accel_incidence(const sesm_ctx* ctx, int r) {
  const AccelOp* A = ctx->acc;
  return (A && r >= 0 && r < A->n_inc) ? &A->inc_prob[r] : nullptr;
}

// Where the near-field items of a single-density forward map run (see
// AccelOp::near_c1).  The tuner times candidate splits on the device and keeps
// the fastest; the candidates give the merge + FFT, y-convolution and
// inverse-FFT launches shares of the items in the ratio of those stages'
// durations on the benched shapes (0.34 : 0.37 : 0.22 of the near-field
// stream's time), scaled by a = 0 .. 1, the first launch keeping the rest
// (a = 0: every item in the first launch); then each launch's share is moved
// by +-6% and +-3% of the items while that helps (coordinate descent).
// Results are cached per grid shape in the context, so a surface of a known
// shape is not timed again.
static void set_split(AccelOp* A, double f_local, double f_merge, double f_yconv) {
  const int n = A->n_chunks;
  auto at = [&](double f) { return std::min(n, std::max(0, (int)std::lround(f * n))); };
  A->near_c1 = at(f_local);
  A->near_c2 = std::max(A->near_c1, at(f_local + f_merge));
  A->near_c3 = std::max(A->near_c2, at(f_local + f_merge + f_yconv));
}

static int choose_near_split(sesm_ctx* ctx) {
  AccelOp* A = ctx->acc;
  const sesm_params& prm = ctx->prm;
  A->tuned_us = 0.0;
  if (prm.near_split < 0) {
    set_split(A, 1.0, 0.0, 0.0);
    return SESM_OK;
  }
  if (prm.near_split == 1) {
    const int* f = prm.split_permille;
    if (f[0] < 0 || f[1] < 0 || f[2] < 0 || f[0] > 1000 || f[1] > 1000 || f[2] > 1000 || f[0] + f[1] + f[2] > 1000)
      return ctx->fail(SESM_EINVAL, "split_permille: each in [0, 1000], sum at most 1000");
    set_split(A, f[0] / 1000.0, f[1] / 1000.0, f[2] / 1000.0);
    return SESM_OK;
  }
  if (prm.near_split != 0) return ctx->fail(SESM_EINVAL, "near_split must be -1, 0 or 1");
  const int64_t key[8] = {ctx->P.N, A->n_chunks, A->n_occ, A->nXH, A->nYH, A->nXV, A->nYV, A->n_groups};
  for (const NearSplit& c : ctx->near_splits)
    if (std::equal(key, key + 8, c.key)) {
      A->near_c1 = c.c1;
      A->near_c2 = c.c2;
      A->near_c3 = c.c3;
      A->tuned_us = c.us;
      return SESM_OK;
    }
  const int N = ctx->P.N;
  int rc;
  cplx *mu = nullptr, *y = nullptr;
  if ((rc = sesm_alloc(ctx, (void**)&mu, sizeof(cplx) * N)) || (rc = sesm_alloc(ctx, (void**)&y, sizeof(cplx) * N)))
    return rc;
  SESM_HIP(hipMemsetAsync(mu, 0x3F, sizeof(cplx) * N, ctx->stream));  // any finite density: times do not depend on it
  hipEvent_t e0, e1;
  SESM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ctx->fail(SESM_EHIP, "hipEventCreate failed");
  }
  const uint32_t kt = ctx->kt_mask;
  ctx->kt_mask = 0;  // the tuner's maps are not counted by the timing classes
  auto trial = [&](double* us) -> int {
    for (int w = 0; w < 2; ++w)
      if (int r = accel_matvec_impl(ctx, mu, y, false)) return r;
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      SESM_HIP(hipEventRecord(e0, ctx->stream));
      for (int t = 0; t < 4; ++t)
        if (int r = accel_matvec_impl(ctx, mu, y, false)) return r;
      SESM_HIP(hipEventRecord(e1, ctx->stream));
      SESM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SESM_HIP(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, 1e3 * ms / 4);
    }
    *us = best;
    return SESM_OK;
  };
  // shares of the items with merge + FFT, y convolution, inverse FFT
  const double wm = 0.34, wy = 0.37, wf = 0.22;
  double best_us = 1e30, best[3] = {0.0, 0.0, 0.0};
  auto try_split = [&](const double* f, double* us) -> int {
    set_split(A, 1.0 - (f[0] + f[1] + f[2]), f[0], f[1]);
    return trial(us);
  };
  // scan the overall share, then refine each launch's share (coordinate descent)
  for (double a : {0.0, 0.3, 0.5, 0.7, 0.85, 1.0}) {  // a = 0: every item in the first launch
    const double f[3] = {a * wm, a * wy, a * wf};
    double us = 0.0;
    if ((rc = try_split(f, &us))) break;
    if (us < best_us) best_us = us, std::copy(f, f + 3, best);
  }
  for (double step : {0.06, 0.03}) {
    for (int i = 0; i < 3 && !rc; ++i)
      for (double sg : {1.0, -1.0}) {
        double f[3] = {best[0], best[1], best[2]};
        f[i] += sg * step;
        if (f[i] < 0.0 || f[0] + f[1] + f[2] > 1.0) continue;
        double us = 0.0;
        if ((rc = try_split(f, &us))) break;
        if (us < best_us) best_us = us, std::copy(f, f + 3, best);
      }
  }
  ctx->kt_mask = kt;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  set_split(A, 1.0 - (best[0] + best[1] + best[2]), best[0], best[1]);
  A->tuned_us = best_us;
  NearSplit c;
  std::copy(key, key + 8, c.key);
  c.c1 = A->near_c1;
  c.c2 = A->near_c2;
  c.c3 = A->near_c3;
  c.us = best_us;
  ctx->near_splits.push_back(c);
  return SESM_OK;
}

// ------------------------------------------------------------------ off-surface field
// The field at points inside the cell grid by the forward map's own stages,
// as the remark closing Sec. 5.7 describes: for a point P in cell c^q,
//   u(P) = (plane-wave expansion of psi^{ni,q}, eq. planewave, at P)
//        + sum over the nodes of the near columns of dx K_dl(P - x_l) mu_l
//        + the completion modes (eq. M_eta) at P,
// where the plane-wave weights come from the boundary values b^q = phi^all
// minus the local corrections of every occupied cell in the near columns
// (eqs. small_convolution, combine_psi_pna) - formed here for any cell,
// occupied or not.  One workgroup per cell holding points.
struct FieldCellArgs {
  int n_x, n_y, n_s, n_e, n_bH, n_bdry, n_eq, n_plw, nXH, nXV, ring, n_cells, N;
  double L, x0, y0;
  const int* tc_cell;      // cells holding points
  const int* tc_off;       // their points: [tc_off[t], tc_off[t + 1]) of the lists below
  const int* tgt;          // point index
  const double* tx;        // point coordinates (x in [x0, x0 + d))
  const double* ty;
  const int* tp;           // quasi-periodic shift (periods) of each listed point
  const int* col_occ_off;  // occupied cells of each column: col_occ[col_occ_off[c] .. col_occ_off[c + 1])
  const int* col_occ;
  const int* col_lo;
  const int* col_w;
  const cplx* W;
  const cplx* dens;
  const cplx* phH;
  const cplx* phV;
  const cplx* pplw;
  const double* dirs;
  const double* x;
  const double* f;
  const double* fp;
  const cplx* mu;
  const cplx* mode_part;
  cplx* u;
};

__global__ __launch_bounds__(256) void k_field_cells(FieldCellArgs A, KParams K) {
  extern __shared__ cplx dyn[];
  __shared__ cplx bv[64];
  __shared__ cplx wv_sh[64];
  __shared__ cplx msum[SESM_MAX_UETA];
  __shared__ cplx red[256];
  const int cell = A.tc_cell[blockIdx.x];
  const int cx = cell % A.n_x, cy = cell / A.n_x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double ccx = A.x0 + (cx + 0.5) * A.L, ccy = A.y0 + (cy + 0.5) * A.L;
  const int npf = (A.n_bdry + A.n_plw + 1) * A.n_plw;
  cplx* pf = dyn;
  const cplx php = cexp_i(K.alpha * K.d);
  stage_copy<10>(pf, A.pplw, npf, threadIdx.x, 256);
  if (wv == 1) {
    for (int t = 0; t < K.nU; ++t) {
      cplx a = cplx{0.0, 0.0};
      for (int c = lane; c < NCH_MODES; c += 64) a += A.mode_part[(int64_t)t * NCH_MODES + c];
      a = wave_sum(a);
      if (lane == 0) msum[t] = a;
    }
  }
  if (threadIdx.x < A.n_bdry) {
    const int b = threadIdx.x;
    cplx val;
    if (b < A.n_bH) {
      const int iy = b / (A.n_s + 1), i = b % (A.n_s + 1);
      int gx = cx * A.n_s + i, Wr = 0;
      if (gx >= A.nXH) { gx -= A.nXH; Wr = 1; }
      val = A.phH[(int64_t)(cy + iy) * A.nXH + gx];
      if (Wr) val = php * val;
    } else {
      const int t = b - A.n_bH, ix = t / (A.n_s - 1), i = 1 + t % (A.n_s - 1);
      int gx = cx + ix, Wr = 0;
      if (gx >= A.nXV) { gx -= A.nXV; Wr = 1; }
      val = A.phV[(int64_t)(cy * A.n_s + i + A.n_e) * A.nXV + gx];
      if (Wr) val = php * val;
    }
    // local corrections of the occupied cells of the near columns (offset o of
    // the source cell, its densities of this boundary point's set)
    const int ns2 = 2 * A.n_eq, lamb = b < A.n_bH ? 0 : 1;
    cplx cs = cplx{0.0, 0.0};
    for (int ox = -A.ring; ox <= A.ring; ++ox) {
      int col = cx + ox;
      const int wr = col < 0 ? -1 : (col >= A.n_x ? 1 : 0);
      col -= wr * A.n_x;
      for (int r = A.col_occ_off[col]; r < A.col_occ_off[col + 1]; ++r) {
        const int rc = A.col_occ[r];
        const int oy = rc / A.n_x - cy;
        const int o = (ox + A.ring) * (2 * A.n_y - 1) + (oy + A.n_y - 1);
        const cplx* Wo = A.W + (int64_t)o * ns2 * A.n_bdry + b;
        const cplx* dv = A.dens + ((int64_t)lamb * A.n_cells + rc) * ns2;
        cplx acc = cplx{0.0, 0.0};
        for (int t = 0; t < ns2; ++t) acc += Wo[(int64_t)t * A.n_bdry] * dv[t];
        cs += wr == 0 ? acc : (wr > 0 ? php : conj(php)) * acc;
      }
    }
    bv[b] = val - cs;
  }
  __syncthreads();
  // plane-wave weights w = V diag(1/sig) U^H b (eq. plwave_QR), one wavefront
  if (wv == 0 && lane < A.n_plw) {
    const cplx* Vs = pf + A.n_bdry * A.n_plw;
    const cplx* isg = Vs + A.n_plw * A.n_plw;
    cplx e = cplx{0.0, 0.0};
    for (int b = 0; b < A.n_bdry; ++b) e += pf[b * A.n_plw + lane] * bv[b];
    red[lane] = isg[lane].re * e;
  }
  __syncthreads();
  if (wv == 0 && lane < A.n_plw) {
    const cplx* Vs = pf + A.n_bdry * A.n_plw;
    cplx w = cplx{0.0, 0.0};
    for (int j = 0; j < A.n_plw; ++j) w += Vs[j * A.n_plw + lane] * red[j];
    wv_sh[lane] = w;
  }
  __syncthreads();
  // the points of the cell, one after another: threads over the near columns'
  // nodes, the plane waves and the modes; a fixed-order block sum
  const int lo = A.col_lo[cx], wdt = A.col_w[cx];
  for (int t = A.tc_off[blockIdx.x]; t < A.tc_off[blockIdx.x + 1]; ++t) {
    const double X = A.tx[t], Y = A.ty[t];
    cplx acc = cplx{0.0, 0.0};
    for (int uu = threadIdx.x; uu < wdt; uu += 256) {
      int l = lo + uu;
      const int wr = l < 0 ? -1 : (l >= A.N ? 1 : 0);
      l -= wr * A.N;
      cplx m = A.mu[l];
      if (wr != 0) m = (wr > 0 ? php : conj(php)) * m;
      acc += (K.dx * m) * sesm_kdl(K, X - (A.x[l] + wr * K.d), Y - A.f[l], A.fp[l]);
    }
    if (threadIdx.x < A.n_plw)
      acc += wv_sh[threadIdx.x] *
             cexp_i(K.k * (A.dirs[2 * threadIdx.x] * (X - ccx) + A.dirs[2 * threadIdx.x + 1] * (Y - ccy)));
    if (threadIdx.x >= 128 && threadIdx.x - 128 < K.nU) {
      const int n = threadIdx.x - 128;
      acc += (exp(-K.Ubi[n] * Y) * cexp_i(K.Ua[n] * X + K.Ubr[n] * Y)) * msum[n];
    }
    const cplx s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) A.u[A.tgt[t]] = cexp_i(K.alpha * K.d * A.tp[t]) * s;
  }
}

AccelGrid sesm_accel_grid(const sesm_ctx* ctx) {
  const AccelOp* A = ctx->acc;
  return AccelGrid{A->x0, A->y0, A->L, A->n_x, A->n_y};
}

int sesm_accel_field_cells(sesm_ctx* ctx, const cplx* mu, int n, const int* idx, const double* px, const double* py,
                           const int* p, cplx* u) {
  AccelOp* A = ctx->acc;
  if (n == 0) return SESM_OK;
  // points by cell
  std::vector<int> cellof(n), order(n);
  for (int t = 0; t < n; ++t) {
    const int cx = std::min(A->n_x - 1, std::max(0, (int)std::floor((px[t] - A->x0) / A->L)));
    const int cy = std::min(A->n_y - 1, std::max(0, (int)std::floor((py[t] - A->y0) / A->L)));
    cellof[t] = cy * A->n_x + cx;
    order[t] = t;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cellof[a] < cellof[b]; });
  std::vector<int> tc_cell, tc_off, tgt(n), tp(n);
  std::vector<double> tx(n), ty(n);
  for (int r = 0; r < n; ++r) {
    const int t = order[r];
    if (tc_cell.empty() || tc_cell.back() != cellof[t]) {
      tc_cell.push_back(cellof[t]);
      tc_off.push_back(r);
    }
    tgt[r] = idx[t];
    tx[r] = px[t];
    ty[r] = py[t];
    tp[r] = p[t];
  }
  tc_off.push_back(n);
  // occupied cells of each column, in increasing cell index
  std::vector<int> occ(A->n_occ);
  SESM_HIP(hipMemcpyAsync(occ.data(), A->occ_cell, sizeof(int) * A->n_occ, hipMemcpyDeviceToHost, ctx->stream));
  SESM_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int> col_occ_off(A->n_x + 1, 0), col_occ;
  for (int c : occ) ++col_occ_off[c % A->n_x + 1];
  for (int c = 0; c < A->n_x; ++c) col_occ_off[c + 1] += col_occ_off[c];
  col_occ.resize(A->n_occ);
  {
    std::vector<int> fill(col_occ_off.begin(), col_occ_off.end() - 1);
    for (int c : occ) col_occ[fill[c % A->n_x]++] = c;
  }
  // device copies (freed before returning; the stream is synchronised)
  const size_t nb = sizeof(int) * (tc_cell.size() + tc_off.size() + 2 * (size_t)n + col_occ_off.size() +
                                   std::max<size_t>(col_occ.size(), 1)) +
                    sizeof(double) * 2 * (size_t)n + sizeof(cplx) * (size_t)ctx->P.N + 256;
  char* buf = nullptr;
  SESM_HIP(hipMalloc((void**)&buf, nb));
  char* cur = buf;
  auto put = [&](const void* src, size_t bytes) -> void* {
    void* d = cur;
    if (bytes) (void)hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, ctx->stream);
    cur += (bytes + 15) / 16 * 16;
    return d;
  };
  cplx* ytmp = (cplx*)cur;
  cur += sizeof(cplx) * (size_t)ctx->P.N;
  FieldCellArgs F;
  F.tc_cell = (const int*)put(tc_cell.data(), sizeof(int) * tc_cell.size());
  F.tc_off = (const int*)put(tc_off.data(), sizeof(int) * tc_off.size());
  F.tgt = (const int*)put(tgt.data(), sizeof(int) * n);
  F.tp = (const int*)put(tp.data(), sizeof(int) * n);
  F.tx = (const double*)put(tx.data(), sizeof(double) * n);
  F.ty = (const double*)put(ty.data(), sizeof(double) * n);
  F.col_occ_off = (const int*)put(col_occ_off.data(), sizeof(int) * col_occ_off.size());
  F.col_occ = (const int*)put(col_occ.data(), sizeof(int) * col_occ.size());
  int rc = accel_matvec_impl(ctx, mu, ytmp, false);  // phi^all grids, densities and mode sums of mu
  if (rc == SESM_OK) {
    F.n_x = A->n_x;
    F.n_y = A->n_y;
    F.n_s = A->n_s;
    F.n_e = A->n_e;
    F.n_bH = A->n_bH;
    F.n_bdry = A->n_bdry;
    F.n_eq = A->n_eq;
    F.n_plw = A->n_plw;
    F.nXH = A->nXH;
    F.nXV = A->nXV;
    F.ring = A->ring;
    F.n_cells = A->n_cells;
    F.N = ctx->P.N;
    F.L = A->L;
    F.x0 = A->x0;
    F.y0 = A->y0;
    F.col_lo = A->col_lo;
    F.col_w = A->col_w;
    F.W = A->W;
    F.dens = A->dens;
    F.phH = A->phH;
    F.phV = A->phV;
    F.pplw = A->pplw;
    F.dirs = A->dirs;
    F.x = ctx->x;
    F.f = ctx->f;
    F.fp = ctx->fp;
    F.mu = mu;
    F.mode_part = A->mode_part;
    F.u = u;
    const size_t lds = sizeof(cplx) * (size_t)(A->n_bdry + A->n_plw + 1) * A->n_plw;
    hipLaunchKernelGGL(k_field_cells, dim3((unsigned)tc_cell.size()), dim3(256), lds, ctx->stream, F,
                       ctx->kparams());
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, std::string("k_field_cells: ") + hipGetErrorString(e));
  }
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (rc == SESM_OK && es != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(es));
  return rc;
}

extern "C" int sesm_diag_accel(sesm_ctx* ctx, const sesm_c64* mu, int32_t which, sesm_c64* out, int64_t out_len) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL || !ctx->acc) return ctx->fail(SESM_EINVAL, "not in accelerated mode");
  if (!mu || !out) return ctx->fail(SESM_EINVAL, "null pointer");
  SESM_HIP(hipSetDevice(ctx->device));
  AccelOp* A = ctx->acc;
  const int N = ctx->P.N;
  cplx* ytmp = nullptr;
  int rc = SESM_OK;
  SESM_HIP(hipMalloc((void**)&ytmp, sizeof(cplx) * N));
  rc = accel_matvec_impl(ctx, (const cplx*)mu, ytmp, true);
  const cplx* src = nullptr;
  int64_t len = 0;
  const int64_t nH = (int64_t)A->nXH * A->nYH, nV = (int64_t)A->nXV * A->nYV;
  switch (which) {
    case 0: src = A->yfar; len = N; break;                                     // far-field contribution at the nodes
    case 1: src = A->phH; len = nH; break;                                     // phi^all on the H grid [nYH][nXH]
    case 2: src = A->phV; len = nV; break;                                     // phi^all on the V grid [nYV][nXV]
    case 3: src = A->dens; len = (int64_t)2 * A->n_cells * 2 * A->n_eq; break; // per-cell densities
    case 4: src = A->bq; len = (int64_t)A->n_occ * A->n_bdry; break;           // boundary values b^q
    case 5: src = A->self_spec; len = A->spec_len; break;                      // kernel spectra
    default: rc = ctx->fail(SESM_EINVAL, "unknown diagnostic buffer");
  }
  if (rc == SESM_OK && out_len < len) rc = ctx->fail(SESM_EINVAL, "output buffer too small");
  if (rc == SESM_OK) {
    hipError_t e = hipMemcpyAsync(out, src, sizeof(cplx) * len, hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) rc = ctx->fail(SESM_EHIP, hipGetErrorString(e));
  }
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(ytmp);
  return rc;
}

extern "C" int sesm_diag_fft(sesm_ctx* ctx, int32_t n, int32_t rows, const sesm_c64* in, sesm_c64* out,
                             int32_t sign) {
  if (!ctx) return SESM_EINVAL;
  if (!in || !out || rows < 1 || (sign != 1 && sign != -1)) return ctx->fail(SESM_EINVAL, "bad FFT arguments");
  FftPlan p;
  if (n < 1 || n > SESM_FFT_MAXN || !sesm_fft_factor(n, &p))
    return ctx->fail(SESM_EINVAL, "FFT length must be 5-smooth and <= 2000");
  SESM_HIP(hipSetDevice(ctx->device));
  std::vector<cplx> tw(n);
  for (int t = 0; t < n; ++t) {
    const double ph = -2.0 * PI * t / n;
    tw[t] = cplx{std::cos(ph), std::sin(ph)};
  }
  cplx* dtw = nullptr;
  SESM_HIP(hipMalloc((void**)&dtw, sizeof(cplx) * n));
  int rc = SESM_OK;
  if (hipMemcpyAsync(dtw, tw.data(), sizeof(cplx) * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
    rc = ctx->fail(SESM_EHIP, "twiddle upload failed");
  } else {
    p.tw = dtw;
    rc = fft_launch(ctx, ctx->stream, sesm_fft_job(p, rows, (const cplx*)in, (cplx*)out, nullptr, nullptr, 1.0),
                    FftJob{}, sign);
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == SESM_OK) rc = ctx->fail(SESM_EHIP, "FFT failed");
  (void)hipFree(dtw);
  return rc;
}

extern "C" int sesm_diag_near(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y) {
  if (!ctx) return SESM_EINVAL;
  if (!ctx->ready) return ctx->fail(SESM_ENOSURF, "no surface");
  if (ctx->P.mode != SESM_MODE_ACCEL || !ctx->acc) return ctx->fail(SESM_EINVAL, "not in accelerated mode");
  if (!mu || !y || (const void*)mu == (const void*)y) return ctx->fail(SESM_EINVAL, "invalid vectors");
  SESM_HIP(hipSetDevice(ctx->device));
  AccelOp* A = ctx->acc;
  const LocalArgs L = local_args(ctx, true);
  hipLaunchKernelGGL(k_local_apply<cplx>, dim3(L.n_chunks), dim3(LOC_NT), 0, ctx->stream, ctx->kparams(), L,
                     (const cplx*)mu, (cplx*)y, A->inc_self);
  SESM_LAUNCH_CHECK();
  return SESM_OK;
}
