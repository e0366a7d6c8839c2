/*
 * sesm.h - C ABI of the MI355X library for 2-D periodic sound-soft (Dirichlet,
 * TE/PEC) scattering with the shifted (multipolar, Wood-anomaly capable)
 * quasi-periodic Green function and shifted-equivalent-source FFT acceleration.
 *
 * Method: O. P. Bruno and M. Maas, "Shifted equivalent sources and FFT
 * acceleration for periodic scattering problems, including Wood anomalies".
 * Section and equation names below refer to that paper.
 *
 * Conventions shared by every entry point
 *  - Units are those of the caller (lengths and wavenumbers consistent).
 *  - Complex numbers are interleaved FP64 pairs (sesm_c64), the memory layout
 *    of torch.complex128 / std::complex<double>.
 *  - Pointers documented as "device" must point to device memory of the
 *    context's GPU, of at least the stated length; "host" pointers are plain
 *    CPU memory.  The library never frees caller memory.
 *  - All device work is enqueued on the stream given to sesm_create; calls
 *    that return results in host memory (sesm_solve's info, sesm_efficiencies,
 *    sesm_get_info) synchronise that stream before returning.
 *  - Return value 0 means success; negative values are SESM_E* codes and
 *    sesm_last_error() returns a human-readable message.  No C++ exception
 *    crosses this interface.  One context must not be used from two threads
 *    at once.
 *  - Quadrature nodes: x_l = l d / N, l = 0..N-1 (the paper numbers them
 *    1..N with x_N = d; by the quasi-periodicity mu_{l+N} = mu_l e^{i alpha d},
 *    eq. (quasiper_disc), this relabels one unknown).  Densities mu_l are the
 *    Nystrom values of eq. (discrete_eq).
 */
#ifndef SESM_H
#define SESM_H

#include <stdint.h>

#if defined(__GNUC__)
#define SESM_API __attribute__((visibility("default")))
#else
#define SESM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define SESM_OK 0
#define SESM_EINVAL (-1)     /* invalid argument or parameter combination      */
#define SESM_ENOSURF (-2)    /* sesm_set_surface has not succeeded yet          */
#define SESM_ENOMEM (-3)     /* device allocation failed                        */
#define SESM_EHIP (-4)       /* HIP runtime error (text in sesm_last_error)     */
#define SESM_ERESONANT (-5)  /* accelerator cell side L is a Dirichlet resonance */
#define SESM_ENOCONV (-6)    /* GMRES did not reach tol; outputs still written   */

#define SESM_MODE_DENSE 0    /* precomputed dense direct operator, Sec. 4.3     */
#define SESM_MODE_ACCEL 1    /* shifted-equivalent-source FFT acceleration, Sec. 5 */

typedef struct sesm_ctx sesm_ctx;

typedef struct {
  double re, im;
} sesm_c64;

/* Profile f(x) = a[0] + sum_{m=1}^{n_modes} a[m] cos(2 pi m x/d) + b[m] sin(2 pi m x/d).
 * a, b: host arrays of length n_modes + 1 (b[0] is ignored). */
typedef struct {
  int32_t n_modes;
  const double* a;
  const double* b;
} sesm_profile;

/* Discretisation parameters.  A zero field selects the documented default. */
typedef struct {
  int32_t N;          /* number of quadrature nodes per period (required, >= 8)          */
  double h;           /* shift of G_j, eq. (shifted_green_function); default pi / k       */
  double c_window;    /* plateau fraction c of the window S_{cA,A}, eq. (na_A); default 0.5 */
  int32_t n_a;        /* singular window radius a = n_a d/N, eq. (dsing_def);
                         default floor(0.8 min(L_cell, d) N / d), at least 8 */
  double gamma_frac;  /* gamma = gamma_frac * a, eq. (S_def); default 0.5                 */
  double eta;         /* completion threshold of U^eta, eq. (M_eta); default 1e-3          */
  int32_t mode;       /* SESM_MODE_DENSE (default) or SESM_MODE_ACCEL                     */
  double L_cell;      /* accelerator cell side L, eq. (L_constr); default 0.5 * 2 pi / k  */
  int32_t n_side;     /* accelerator: equivalent-source grid intervals per cell side      */
  int32_t n_ext;      /* accelerator: extra equivalent-source points beyond each corner;
                         0 selects 1, a negative value selects none; the points per side,
                         n_side + 1 + 2 n_ext, must not exceed 16 (SESM_EINVAL)           */
  int32_t n_coll;     /* accelerator: collocation points per side of the 3L square, eq. (eq_source_point) */
  int32_t n_plw;      /* accelerator: plane waves per cell, eq. (planewave)               */
  int32_t near_ring;  /* accelerator: columns on each side of a cell treated directly
                         (near field); default 1, at most 3                              */
  int32_t near_split; /* accelerator: where the near-field work items of a single-density
                         forward map run.  0 (default): a split chosen by timing candidate
                         splits once per grid shape (cached in the context); 1: the split
                         given by split_permille; -1: all of them in the first launch.
                         Every split gives the same results bit for bit.              */
  int32_t split_permille[3]; /* near_split = 1: thousandths of the items in the first
                         launch, with merge + forward FFT, with the y convolution (the
                         inverse FFT takes the rest); each in [0, 1000], sum <= 1000     */
  int32_t mixed;      /* accelerator: 1 also builds the FP32 copy of the EqSources
                         operators (eq. eq_source_point) used by mixed-precision solves
                         (SESM_SOLVE_MIXED); 0 (default) does not                      */
  int32_t table;      /* accelerator kernel tables (the only use of G~_j, Sec. 5.5.1):
                         0 (default): windowed spatial lattice sums (eq. Gq_limit) on
                         every row of the difference grids; 1: hybrid (Sec. 3.2, Remark
                         large_FFT_eval): rows whose height Y keeps a distance
                         delta > 0 from every shifted pole row Y = -m h take the
                         exponentially convergent spectral series (eq.
                         shifted_quasi_per_rayleigh, in the form of eq. betan_taylor
                         at and around Wood anomalies; the exact G~_j, no window),
                         truncated where e^{-|beta_n| delta} < e^{-42} (at most
                         40000 orders); the other rows keep the windowed sums,
                         with a window 8 times as wide (their window error would
                         otherwise jump between neighbouring rows, and at Wood
                         anomalies, where it decays only like A^{-3.5}, the
                         cells' plane-wave fits amplify such jumps).
                         Needs j >= 1 and the accelerated mode.                   */
  int32_t batch_mfma; /* accelerator: 1 applies the near field of batched forward maps
                         (sesm_matvec_batch, sesm_solve_batch and the incidence-set
                         calls) to groups of up to eight densities on the FP64 matrix
                         cores (one pass over the stored blocks per eight densities);
                         the sums are then formed in another order than in
                         sesm_matvec, so batch members agree with single forward maps
                         to rounding, not bit for bit.  0 (default): four densities
                         per pass on the vector units, bit for bit.               */
  int32_t adjoint;    /* dense mode: 1 also forms the derivative matrices dA/dY and
                         dA/df' of the operator entries (sesm_shape_gradient) in the
                         same pass over the lattice sums as the operator itself, and
                         keeps them with the surface (2 N^2 more complex values), so
                         that sesm_shape_gradient does not form them again; 0
                         (default): sesm_shape_gradient forms them on each call.
                         SESM_EINVAL with the accelerated mode.                   */
} sesm_params;

typedef struct {
  int32_t iters;          /* Krylov iterations performed            */
  double rel_residual;    /* final true relative residual ||b - A mu|| / ||b||, with
                             A mu formed by one more forward map after the last cycle */
  int32_t converged;      /* 1 if rel_residual (the true one) <= tol */
  int32_t column_mismatches; /* Hessenberg columns whose copy streamed to the host
                                during a cycle differed from the device's (the
                                update of mu always uses the device's); 0 expected */
  double est_residual;    /* the Givens (least-squares) estimate of the relative
                             residual at the end of the last Krylov cycle      */
  int32_t residual_restarts; /* extra Krylov cycles started because the true
                                residual was above tol while the estimate was not */
  int32_t reserved_i;
} sesm_solve_info;

/* flags of sesm_solve / sesm_solve_batch */
#define SESM_SOLVE_X0 1  /* mu holds the initial guess x0 on entry (warm start) */
#define SESM_SOLVE_MIXED 2 /* mixed precision: FP64 iterative refinement (true residuals
                              with the FP64 forward map) around inner GMRES solves with an
                              FP32 Krylov basis and the mixed-precision map (EqSources
                              operators in FP32, all sums and the near field in FP64);
                              needs a surface set up with sesm_params.mixed = 1.
                              residual_restarts then counts the refinement steps. */
#define SESM_SOLVE_ADJOINT 4 /* solve the conjugate-transpose system (1/2 I + D^dx)^H mu = b
                              (dense mode; b must be given): the adjoint densities of
                              sesm_shape_gradient. */

/* Read-only description of the discretisation chosen by sesm_set_surface. */
typedef struct {
  int32_t N;
  int32_t n_a;
  double dx, a, gamma, h, A_len;
  int32_t mode;
  int32_t n_eta;              /* |U^eta|                                    */
  int32_t U_eta[16];          /* its first 16 members                       */
  int32_t n_first, n_count;   /* propagating orders n_first..n_first+n_count-1 */
  /* accelerator geometry (zeros in dense mode) */
  int32_t n_x, n_y, n_cells_occupied, stencil_rows;
  double L, y0, delta;
  int64_t near_entries;       /* stored near-field entries (accelerated mode) */
  int64_t device_bytes;       /* device memory held by the context (including blocks
                                 kept from an earlier surface for reuse)      */
  int32_t near_items[4];      /* near-field work items per launch of a single-density
                                 forward map: first launch, merge + FFT, y convolution,
                                 inverse FFT                                   */
  double near_tuned_us;       /* forward-map time of the chosen split when the tuner
                                 measured it (0 otherwise)                     */
  int32_t spectral_rows[2];   /* hybrid tables: rows of the horizontal and vertical
                                 difference grids taken from the spectral series
                                 (of 2 n_rows - 1 each; 0 with windowed tables)   */
} sesm_surface_info;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL
 * selects the default stream).  *out receives the context.  Debug aid: when
 * the environment variable SESM_POISON_ALLOC is set (and not "0") at this
 * call, every device buffer the context allocates is first filled with 0xFF
 * bytes (NaN doubles), so that a read before the first write shows up as NaN
 * in the results. */
SESM_API int sesm_create(sesm_ctx** out, int device, void* hip_stream);

/* Release a context and every device buffer it owns.  NULL is accepted. */
SESM_API int sesm_destroy(sesm_ctx* ctx);

/* Algorithm 2 (Initialization): set up the surface and precompute every
 * operator table.  d: period; k: wavenumber; alpha: Bloch wavenumber
 * (alpha = k sin theta, Sec. 2); j: shift order of G_j; A_periods: window
 * half-width A of S_{cA,A} in periods (eq. na_A).  params may be NULL only if
 * N is given through a non-NULL struct, so in practice it is required.
 * Rejects |alpha| > k, a >= d, (accelerated mode) a >= L or a resonant cell
 * side (Remark non-resonant), and non-finite profile values. */
SESM_API int sesm_set_surface(sesm_ctx* ctx, const sesm_profile* profile, double d, double k,
                     double alpha, int32_t j, double A_periods, const sesm_params* params);

/* Algorithm 3 (forward map): y = (1/2 I + D^dx) mu, eq. (discrete_eq).
 * mu, y: device arrays of N sesm_c64; they must not overlap. */
SESM_API int sesm_matvec(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y);

/* Forward maps of several densities with the operator of the current
 * surface: y_r = (1/2 I + D^dx) mu_r, r = 0..nrhs-1, eq. (discrete_eq).
 * Density r is the device array mu + r ld_mu of N sesm_c64, output r is
 * y + r ld_y (ld_mu, ld_y >= N, in elements); the span of the densities must
 * not overlap that of the outputs.  Densities whose incident Bloch
 * wavenumbers differ by multiples of 2 pi / d share this operator: it depends
 * on alpha only through e^{i alpha d} (eq. shifted_periodic_green_function)
 * and the set {alpha_n} (eqs. alpha_beta_def, M_eta).  In accelerated mode groups of up to four densities
 * share one pass over the near-field blocks and the equivalent-source
 * projections (Algorithm 3), and the results equal those of sesm_matvec
 * bit for bit; in dense mode the densities are applied one at a time.
 * nrhs = 0 does nothing; nrhs < 0, ld below N, overlap or NULL pointers give
 * SESM_EINVAL.  The first accelerated call allocates the per-density
 * buffers of four densities (owned by the surface).  Kernel timing records
 * each later stage once per group of up to four densities (bytes of all of
 * them), not the shared first launch. */
SESM_API int sesm_matvec_batch(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* mu, int64_t ld_mu, sesm_c64* y,
                               int64_t ld_y);

/* Right-hand side of eq. (discrete_eq): b_l = -u^inc(x_l, f(x_l)) with
 * u^inc = exp(i (alpha x - beta y)), beta = sqrt(k^2 - alpha^2) (Sec. 2).
 * b: device array of N sesm_c64. */
SESM_API int sesm_rhs(sesm_ctx* ctx, sesm_c64* b);

/* Right-hand side of member p of the surface's Bloch class: the incidence
 * with alpha_p = alpha + 2 pi p / d, beta_p = sqrt(k^2 - alpha_p^2), which sees
 * the same operator (eqs. shifted_periodic_green_function, alpha_beta_def);
 * b_l = -exp(i (alpha_p x_l - beta_p f(x_l))).  p = 0 gives sesm_rhs.  b:
 * device array of N sesm_c64.  SESM_EINVAL if |alpha_p| >= k. */
SESM_API int sesm_rhs_bloch(sesm_ctx* ctx, int32_t p, sesm_c64* b);

/* Algorithm 1: GMRES solve of (1/2 I + D^dx) mu = b.  b: device array of N
 * (NULL selects the incident-field right-hand side of sesm_rhs).  mu: device
 * array of N; with SESM_SOLVE_X0 in flags it holds the initial guess x0 on
 * entry (in: x0, out: solution), otherwise the iteration starts from zero and
 * mu is output only.  tol: relative residual; max_iter: iteration cap (over
 * all cycles); restart: Krylov dimension of a cycle (0 = max_iter, i.e.
 * unrestarted; at most 4000).  When a cycle's least-squares estimate reaches
 * tol, the true residual b - A mu is formed with one more forward map; if it
 * is still above tol and iterations remain, a new cycle starts from it (the
 * restart step) - unless this is already such a restart and the true
 * residual fell by less than half, which means it has reached the level the
 * forward map's own rounding allows (the accelerated map is linear only up to
 * its rounding noise, ~1e-12 relative; the attainable true residual is about
 * that noise times |mu| / |b| times the square root of the Krylov dimension).
 * converged and rel_residual report the true residual.
 * info: host struct, may be NULL.  Returns SESM_ENOCONV if tol was not
 * reached (mu and info still hold the last iterate). */
SESM_API int sesm_solve(sesm_ctx* ctx, const sesm_c64* b, sesm_c64* mu, double tol, int32_t max_iter,
               int32_t restart, int32_t flags, sesm_solve_info* info);

#define SESM_MAX_BATCH 64  /* right-hand sides per sesm_solve_batch call */

/* Algorithm 1 for several right-hand sides with the operator of the current
 * surface (for instance the incidences of one Bloch class, see
 * sesm_matvec_batch): one unrestarted GMRES per right-hand side, run in
 * lockstep so that every Arnoldi step applies the operator to all active
 * systems with one batched forward map (Algorithm 3).  Right-hand side r is
 * the device array b + r ld_b of N sesm_c64, solution r is mu + r ld_mu
 * (with SESM_SOLVE_X0 in flags it holds that system's initial guess on entry,
 * otherwise it is output only and the iteration starts from zero); ld_b,
 * ld_mu >= N and the two spans must not overlap.  A system leaves the batch
 * once its least-squares estimate reaches tol; the true residuals are then
 * formed with one batched forward map, and a system whose true residual is
 * still above tol continues alone with restarted cycles (sesm_solve with a
 * warm start) while iterations remain.  Each solution equals that of
 * sesm_solve(b_r, restart = 0, same flags) with the same tol and max_iter bit
 * for bit.  0 <= nrhs <= SESM_MAX_BATCH,
 * 1 <= max_iter <= 4000.  info: host array of nrhs records, may be NULL.
 * The call allocates its work space (nrhs (max_iter + 1) N complex values for
 * the bases, plus small buffers) and returns it to the context's pool at the
 * end.  Returns SESM_ENOCONV if any system missed tol (all outputs still
 * written). */
SESM_API int sesm_solve_batch(sesm_ctx* ctx, int32_t nrhs, const sesm_c64* b, int64_t ld_b, sesm_c64* mu,
                              int64_t ld_mu, double tol, int32_t max_iter, int32_t flags, sesm_solve_info* info);

/* ---- Incidence sets: several incidences on one surface and wavenumber ----
 *
 * The accelerated operator depends on the incidence only through the Bloch
 * wavenumber alpha: the phase e^{-i alpha d p} of the lattice sums (eq.
 * shifted_periodic_green_function, eq. Gq_limit), the phase e^{i alpha d} of
 * source images across the period boundary, and the completion set U^eta
 * with its modes (eq. M_eta).  The near-field blocks, the EqSources
 * operators (eq. eq_source_point), the local-correction matrices
 * (eq. small_convolution) and the plane-wave factors (eq. plwave_QR) do not
 * depend on alpha.  An incidence set keeps one copy of those and, per
 * member, only the alpha-dependent tables (kernel spectra, twist factors,
 * completion modes; about 3 MB per member at N = 32768).  Accelerated mode
 * only.  A new sesm_set_surface clears the set. */
#define SESM_MAX_INCIDENCES 4096

/* Set the incidence set: n Bloch wavenumbers alpha_host[0..n-1] (host,
 * |alpha| < k each; n = 0 clears the set).  Builds the members' tables
 * (their windowed lattice sums: about 1 ms each at N = 32768).  The surface's
 * own incidence (sesm_set_surface's alpha) is unaffected. */
SESM_API int sesm_set_incidences(sesm_ctx* ctx, int32_t n, const double* alpha_host);

/* Right-hand side of member r: b_l = -exp(i (alpha_r x_l - beta_r f(x_l))).
 * b: device array of N sesm_c64. */
SESM_API int sesm_rhs_incidence(sesm_ctx* ctx, int32_t r, sesm_c64* b);

/* Forward maps (Algorithm 3) of members r0 .. r0 + nrhs - 1: density i
 * (device array mu + i ld_mu of N) with the operator of member r0 + i, into
 * y + i ld_y.  Groups of up to four densities share one pass over the
 * near-field blocks and EqSources operators; each later stage is one launch
 * per group with the members' own tables.  Same argument rules as
 * sesm_matvec_batch; member indices beyond the set give SESM_EINVAL. */
SESM_API int sesm_matvec_incidences(sesm_ctx* ctx, int32_t r0, int32_t nrhs, const sesm_c64* mu, int64_t ld_mu,
                                    sesm_c64* y, int64_t ld_y);

/* Algorithm 1 for members r0 .. r0 + nrhs - 1 in lockstep (as
 * sesm_solve_batch): system i has the operator of member r0 + i and the
 * right-hand side b + i ld_b, or, with b = NULL, that member's incident
 * field (sesm_rhs_incidence).  mu, flags, tol, max_iter and info as in
 * sesm_solve_batch (nrhs <= SESM_MAX_BATCH). */
SESM_API int sesm_solve_incidences(sesm_ctx* ctx, int32_t r0, int32_t nrhs, const sesm_c64* b, int64_t ld_b,
                                   sesm_c64* mu, int64_t ld_mu, double tol, int32_t max_iter, int32_t flags,
                                   sesm_solve_info* info);

/* Efficiencies and energy balance (as sesm_efficiencies) of a density mu
 * solved for member r: the Rayleigh coefficients with alpha_r, its orders
 * and completion set. */
SESM_API int sesm_efficiencies_incidence(sesm_ctx* ctx, int32_t r, const sesm_c64* mu, int32_t* n_first,
                                         int32_t* n_count, double* e_host, int32_t e_capacity, double* energy_error);

/* Efficiencies e_n = (beta_n / beta) |B_n|^2 of the propagating orders
 * (Sec. 2) and the energy-balance error eps = 1 - sum e_n, eq. (energy_error).
 * B_n are the Rayleigh coefficients of the representation
 * eq. (eq:int_eq_dirichlet) above the surface (spectral series
 * eq. (shifted_periodic_green_function_spectral) plus M^eta), by the
 * trapezoidal rule.  mu: device array of N.  On return *n_first, *n_count
 * describe the orders n_first..n_first+n_count-1; e_host (host, capacity
 * e_capacity) receives min(n_count, e_capacity) values; energy_error (host)
 * may be NULL.  Synchronises the stream. */
SESM_API int sesm_efficiencies(sesm_ctx* ctx, const sesm_c64* mu, int32_t* n_first, int32_t* n_count,
                      double* e_host, int32_t e_capacity, double* energy_error);

/* Rayleigh coefficients B_n for the n_orders integer orders in orders_host
 * (host array); B_host (host, n_orders entries) receives them.  Same
 * formula as sesm_efficiencies.  Synchronises the stream. */
SESM_API int sesm_rayleigh(sesm_ctx* ctx, const sesm_c64* mu, const int32_t* orders_host, int32_t n_orders,
                  sesm_c64* B_host);

/* sesm_rayleigh for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same Rayleigh coefficients (same kernel, same values bit for bit), with
 * the per-order constants and the results kept in a fixed device array of the
 * library instead of the context's buffers.  The call allocates and frees no
 * device memory.  The array holds SESM_RAYLEIGH_NOALLOC_MAX orders (256 KB on
 * every GPU the library runs on, held until the process ends); more orders
 * give SESM_EINVAL.  All contexts on one GPU share that array and each call
 * leaves its results there: calls that overlap in time on one GPU (other
 * threads or streams) race and must be serialised by the caller.  mu: device
 * array of N; orders_host, B_host: host arrays of n_orders.  Synchronises the
 * stream. */
#define SESM_RAYLEIGH_NOALLOC_MAX 4096
SESM_API int sesm_rayleigh_noalloc(sesm_ctx* ctx, const sesm_c64* mu, const int32_t* orders_host, int32_t n_orders,
                                   sesm_c64* B_host);

/* Scattered field off the surface: u(P) of eq. (eq:int_eq_dirichlet) for the
 * density mu (device, N sesm_c64; e.g. a solution of sesm_solve) at n points
 * P_t = (xy[2t], xy[2t + 1]) (device array of 2n doubles, any x: the field is
 * alpha-quasi-periodic), written to u (device, n sesm_c64).  The points must
 * lie off the curve y = f(x) (several dx away for full accuracy: the
 * trapezoidal rule's error falls like exp(-2 pi distance / dx)); below the
 * curve the result is the representation's value, not a physical field.
 * Routes (per point):
 *  - accelerated mode, points inside the accelerator's cell grid
 *    (y0 <= y < y0 + n_y L, sesm_get_info): one forward map of mu and then,
 *    per cell holding points, the plane-wave expansion of the cell's far field
 *    fitted to its boundary values (eq. planewave), the direct sum over the
 *    nodes of the near columns and the completion modes - the "slightly
 *    modified Algorithm 3" of the remark closing Sec. 5.7;
 *  - accelerated mode, points at least L/4 above max f: the Rayleigh
 *    expansion sum_n B_n e^{i alpha_n x + i beta_n y} (Sec. 2; the exact
 *    lattice sum, no window), with every order up to where the terms fall
 *    below e^{-40};
 *  - all other points, and all points in dense mode: the trapezoidal rule of
 *    the windowed lattice sums over all nodes plus the completion modes
 *    (cost O(N A/d j) per point).
 * The grid and direct routes share the operator's window S_{cA,A}; the
 * Rayleigh route is its A -> infinity limit (they differ by the window's
 * truncation error).  Allocates and frees a temporary device buffer;
 * synchronises the stream.  SESM_EINVAL for non-finite coordinates. */
SESM_API int sesm_field(sesm_ctx* ctx, const sesm_c64* mu, int32_t n, const double* xy, sesm_c64* u);

/* Adjoint map (dense mode): y = (1/2 I + D^dx)^H mu, the conjugate transpose of
 * the operator of eq. (discrete_eq).  mu, y: device arrays of N sesm_c64, not
 * overlapping.  Enqueued on the context's stream. */
SESM_API int sesm_matvec_adjoint(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y);

/* Efficiency objective and its adjoint right-hand side (both modes).  For the
 * density mu (device, N) of the current surface and weights w[t] of the
 * propagating orders n = n_first + t (host, n_w = n_count values, the order of
 * sesm_efficiencies): *J = sum_n w_n e_n with e_n = (beta_n / beta) |B_n|^2
 * (Sec. 2; B_n = sum_l c_n(l) mu_l as in sesm_rayleigh), and
 * rhs = conj(g), g_l = sum_n w_n (beta_n / beta) conj(B_n) c_n(l) (device, N):
 * the right-hand side of the adjoint solve (SESM_SOLVE_ADJOINT) whose solution
 * sesm_shape_gradient takes.  J may be NULL.  Synchronises the stream. */
SESM_API int sesm_objective_adjoint_rhs(sesm_ctx* ctx, const sesm_c64* mu, const double* w, int32_t n_w,
                                        sesm_c64* rhs, double* J);

/* Shape gradient (dense mode) of the objective J of sesm_objective_adjoint_rhs
 * with respect to the profile's Fourier coefficients (sesm_profile a[m], b[m],
 * m = 0..n_modes): for the solution mu of the direct problem and the adjoint
 * density nu (solution of SESM_SOLVE_ADJOINT with the right-hand side of
 * sesm_objective_adjoint_rhs),
 *   dJ/dtheta = 2 Re[ sum_n a_n sum_l (dc_n(l)/dtheta) mu_l
 *                     + sum_i conj(nu_i) (db_i/dtheta - sum_l (dA_il/dtheta) mu_l) ],
 * a_n = w_n (beta_n / beta) conj(B_n), with the entry derivatives taken
 * analytically (the double-layer kernel and its windowed lattice sum, eq.
 * DAdx_def; the singular split of eq. local_mat with K_s of eq. ks_def and the
 * log weights; K_r(x, x); the completion modes of eq. M_eta).  grad_a,
 * grad_b: host arrays of n_modes + 1 doubles (grad_b[0] = 0).  The derivative
 * matrices dA/dY, dA/df' are those the set-up kept (sesm_params.adjoint = 1),
 * else formed for the call in two N x N complex work matrices; synchronises
 * the stream. */
SESM_API int sesm_shape_gradient(sesm_ctx* ctx, const sesm_c64* mu, const sesm_c64* nu, const double* w,
                                 int32_t n_w, int32_t n_modes, double* grad_a, double* grad_b);

/* Describe the current discretisation (host struct).  Returns SESM_ENOSURF
 * before a successful sesm_set_surface. */
SESM_API int sesm_get_info(const sesm_ctx* ctx, sesm_surface_info* info);

/* Message of the last failing call on ctx ("" if none).  Never NULL. */
SESM_API const char* sesm_last_error(const sesm_ctx* ctx);

/* Diagnostic (accelerated mode): apply the forward map to mu (device, N) and
 * copy one intermediate result into out (device, out_len sesm_c64):
 *   which = 0: far-field (non-intersecting) contribution at the N nodes;
 *   1: phi^all on the horizontal grid, row-major [n_y + 1][n_x n_s]
 *      (eq. large_convolution_per_grid);  2: phi^all on the vertical grid
 *      [n_y n_s + 1 + 2 n_ext][n_x];  3: per-cell equivalent-source densities
 *      [2 sets][n_x n_y cells][xi (n_eq), zeta (n_eq)] (eq. eq_source_point);
 *   4: the boundary values b^q of the occupied cells (phi^all minus the local
 *      corrections, eqs. psi_na_sum and combine_psi_pna), [occupied cell in
 *      increasing cell index][boundary point: the 2 (n_side + 1) points of the
 *      bottom then top side, then the 2 (n_side - 1) inner points of the left
 *      then right side];
 *   5: the kernel spectra of the surface's own incidence: the x-transforms
 *      (sum_t tab[t] e^{-2 pi i b t / nX}) of the twisted tables
 *      G~_j(X, Y) e^{-i alpha X} of the monopole then the dipole kernel, for
 *      the horizontal grid [2][2 (n_y + 1) - 1][n_x n_s] followed by the
 *      vertical grid [2][2 (n_y n_s + 1 + 2 n_ext) - 1][n_x]; row r holds
 *      height Y = (r - n_rows + 1) hy (mu is not used).
 * Synchronises the stream.  Returns SESM_EINVAL if out_len is too small. */
SESM_API int sesm_diag_accel(sesm_ctx* ctx, const sesm_c64* mu, int32_t which, sesm_c64* out, int64_t out_len);

/* Diagnostic (accelerated mode): y = the direct near-field part of the forward
 * map alone - the intersecting interactions of eq. (final_correction_0), the
 * singular part eq. (local_mat) and 1/2 I, for the sources of the cells in
 * the near columns - as one kernel launch (the near-field work items of the
 * forward map's first kernel) on the context's stream (no synchronisation).  mu, y: device arrays of N sesm_c64, not overlapping. */
SESM_API int sesm_diag_near(sesm_ctx* ctx, const sesm_c64* mu, sesm_c64* y);

/* Diagnostic: the library's own FFT (the transform of the periodic grid
 * direction, Sec. 5.5.1) on caller data: out[r][j] = sum_t in[r][t]
 * exp(sign 2 pi i j t / n) for rows r < rows.  in, out: device arrays of
 * rows x n sesm_c64, row-major (in-place allowed).  n must be 5-smooth and at
 * most 2000; sign is +1 or -1.  Synchronises the stream. */
SESM_API int sesm_diag_fft(sesm_ctx* ctx, int32_t n, int32_t rows, const sesm_c64* in, sesm_c64* out,
                           int32_t sign);

/* Diagnostic: evaluate the library's FP64 Hankel functions H0^(1)(x),
 * H1^(1)(x) (used by every Green-function kernel, eq. free_space) at n
 * points.  x: device array of n doubles (x > 0); h0, h1: device arrays of n
 * sesm_c64.  Enqueued on the context's stream. */
SESM_API int sesm_diag_hankel(sesm_ctx* ctx, const double* x, int32_t n, sesm_c64* h0, sesm_c64* h1);

/* Diagnostic: evaluate the library's own phase factor e^{it} (reduction
 * modulo pi/2 and Taylor polynomials; used for the plane-wave exponentials of
 * eq. planewave) at n points, valid for |t| < 1e5.  t: device array of n
 * doubles; out: device array of n sesm_c64.  Enqueued on the context's stream. */
SESM_API int sesm_diag_cexp(sesm_ctx* ctx, const double* t, int32_t n, sesm_c64* out);

/* Per-kernel timing.  Bit i of a mask selects kernel class i. */
enum {
  SESM_KT_LOCAL = 0,  /* near-field GEMV (intersecting + singular + 1/2 I), cell
                         equivalent-source densities (EqSources) and the partial
                         sums of the completion modes: one launch                   */
  SESM_KT_MERGE = 1,  /* merge onto the periodic grids fused with their forward FFT
                         along x (1 per forward map)                              */
  SESM_KT_FFT = 2,    /* inverse FFT along x of both grids + untwist (1 per map)    */
  SESM_KT_YCONV = 3,  /* convolution along y per x-frequency, both grids, and the
                         local corrections (1 per map)                            */
  SESM_KT_CELLS = 4,  /* boundary values, plane-wave fit, surface values, modes     */
  SESM_KT_DOTS = 5,   /* GMRES: dot products of the Krylov basis with u and A u      */
  SESM_KT_UPDATE = 6, /* GMRES: partial sums of the two basis updates (+ H s)        */
  SESM_KT_GEMV = 7,   /* dense mode: GEMV with the stored operator                   */
  SESM_KT_COUNT = 8
};

typedef struct {
  char name[40];     /* kernel name                                                  */
  int64_t launches;  /* launches timed (bracketed) since sesm_timing_enable           */
  double total_ms;   /* sum of their durations (a HIP event pair around each launch,
                        recorded on the stream the kernel runs on)                    */
  double bytes;      /* sum of their algorithmic HBM bytes: every input array read
                        once and every output array written once                      */
} sesm_kernel_stat;

/* Start timing the kernel classes selected by mask, clearing all counters
 * (mask 0 stops timing).  Every every-th launch of a selected class (1: each
 * launch) is bracketed by HIP events; other launches are not touched, so a
 * sparse sample keeps the brackets' own cost out of a timed region.
 * Enqueues nothing itself.  every < 1 is rejected (SESM_EINVAL). */
SESM_API int sesm_timing_enable(sesm_ctx* ctx, uint32_t mask, int32_t every);

/* Synchronise every stream the timed launches ran on and store SESM_KT_COUNT
 * records (host array, capacity n_stats >= SESM_KT_COUNT), one per class in
 * class order.  Counters keep accumulating until the next sesm_timing_enable. */
SESM_API int sesm_timing_read(sesm_ctx* ctx, sesm_kernel_stat* stats, int32_t n_stats);

#ifdef __cplusplus
}
#endif

#endif /* SESM_H */
