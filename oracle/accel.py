"""Accelerated forward map, Algorithm 3 (oracle; test infrastructure).

Plain NumPy restatement of Sec. 5, step by step, for per-stage parity of the
GPU accelerator and to pin it against the dense direct operator (dense.py),
which it approximates.

Geometry (Sec. 5.1).  Square cells of side L = d / n_x (n_x the smallest
5-smooth integer >= d / L_requested, at least 3), half-open
(a1, b1] x (a2, b2] (Remark cell_def), columns starting at x0 = -dx/2 so that
each node x_l = l dx lies in exactly one column of the reference period, rows
from y0 (below min f) to y0 + n_y L (above max f).

Equivalent sources (Sec. 5.2, eq. eq_mesh).  Grid spacing delta = L / n_s.
Horizontal set of a cell: the points x0 + (c n_s + i) delta, i = -n_e..n_s+n_e,
on its bottom and top sides; vertical set: y0 + (t n_s + i) delta on its left
and right sides.  Monopoles and dipoles whose normals are the fixed directions
(0, 1) (horizontal sets) and (1, 0) (vertical sets), so that densities of
different cells at a shared grid point add (eq. sum_eqsources).  Densities
solve the least-squares problem eq. (eq_source_point) with n_coll collocation
points per side of the 3L square S_q (eq. Sq_notation) around the cell.

Near/far split.  The paper's intersecting set L(q) (eq. small_convolution) is
replaced by a superset: all cells of the three columns q_x - 1, q_x, q_x + 1.
For every other cell r, c^q lies outside the 3L square of r and all of its
downward shifts (eq. S_jq_hat), so the shifted equivalent-source
representation (eq. psi_jr_approx) is valid for it; on a graph surface the
direct near field then is one cyclic band of nodes per column.

Global convolution (Sec. 5.5.1).  Kernel = windowed shifted lattice sum
G~^{q,A}_j (eq. Gq_limit with the Bloch phase) and its normal derivative,
punctured term by term where a term is singular (the reading of eq. phi_def).
x is circular after the twist exp(-i alpha x) (quasi-periodicity, Remark
large_FFT_eval); y is a direct (linear) convolution.

Local correction (Sec. 5.5.2) uses the free-space Phi_j with the same
puncture; plane waves (eq. planewave, plwave_QR) reconstruct the
non-intersecting field inside each cell from its boundary grid values
(corners take the horizontal value, eq. combine_psi_pna).
"""
import numpy as np
from scipy.linalg import solve_triangular
from scipy.special import hankel1

from . import greens, rayleigh


# ---------------------------------------------------------------- geometry
def smooth5_at_least(n):
    """Smallest integer >= n whose prime factors are 2, 3, 5 (the number of
    cells per period sets the length of the periodic convolution)."""
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


class Geometry:
    """Cell grid of Sec. 5.1.  Defaults: n_x the smallest 5-smooth count with
    L close to the requested side, rows centred on the surface's height range.
    n_x (any count >= 3, no FFT-length restriction here) and rows_below (extra
    rows added under the surface, which moves the row grid against the
    surface by whole cells) override those choices; ring sets the near
    columns on each side and coll_ring the collocation square (2 coll_ring + 1) L."""

    def __init__(self, disc, L=0.5, n_s=10, n_e=1, n_coll=60, n_plw=32, ring=1, coll_ring=1, n_x=None,
                 rows_below=0):
        self.disc = disc
        self.ring = ring
        self.coll_ring = coll_ring
        d = disc.d
        self.n_x = int(n_x) if n_x else smooth5_at_least(max(3, int(round(d / L))))
        self.L = d / self.n_x
        self.n_s, self.n_e, self.n_coll, self.n_plw = n_s, n_e, n_coll, n_plw
        self.delta = self.L / n_s
        self.x0 = -0.5 * disc.dx
        fmin, fmax = float(np.min(disc.f)), float(np.max(disc.f))
        self.n_y = int(np.floor((fmax - fmin) / self.L)) + 1 + int(rows_below)
        self.y0 = 0.5 * (fmin + fmax) - 0.5 * (self.n_y - rows_below) * self.L - rows_below * self.L
        # cell of every node, (a, b] convention
        self.cx = np.ceil((disc.x - self.x0) / self.L).astype(np.int64) - 1
        self.cy = np.ceil((disc.f - self.y0) / self.L).astype(np.int64) - 1
        assert np.all((self.cx >= 0) & (self.cx < self.n_x) & (self.cy >= 0) & (self.cy < self.n_y))
        self.cell = self.cy * self.n_x + self.cx
        self.cells = np.unique(self.cell)           # occupied cells
        self.members = {c: np.nonzero(self.cell == c)[0] for c in self.cells}
        self.n_side = n_s + 1 + 2 * n_e              # points per (extended) side
        self.n_eq = 2 * self.n_side                  # per set (H or V)

    def cell_origin(self, c):
        return self.x0 + (c % self.n_x) * self.L, self.y0 + (c // self.n_x) * self.L

    def eq_points(self, lam):
        """Equivalent-source points relative to the cell's lower-left corner,
        as integer grid offsets (ix, iy) in units (delta, L) for H and
        (L, delta) for V, plus positions."""
        i = np.arange(-self.n_e, self.n_s + self.n_e + 1)
        if lam == "H":
            ix = np.concatenate([i, i])
            iy = np.concatenate([np.zeros_like(i), np.ones_like(i)])
            pos = np.stack([ix * self.delta, iy * self.L], 1)
        else:
            ix = np.concatenate([np.zeros_like(i), np.ones_like(i)])
            iy = np.concatenate([i, i])
            pos = np.stack([ix * self.L, iy * self.delta], 1)
        return ix, iy, pos

    def collocation(self):
        """n_coll equispaced points per side of the (2 coll_ring + 1) L square
        around the cell (relative to the cell's lower-left corner)."""
        L, n, r = self.L, self.n_coll, self.coll_ring
        t = (np.arange(n) + 0.5) / n * (2 * r + 1) * L - r * L
        lo, hi = -r * L, (r + 1) * L
        pts = [np.stack([t, np.full(n, lo)], 1), np.stack([t, np.full(n, hi)], 1),
               np.stack([np.full(n, lo), t], 1), np.stack([np.full(n, hi), t], 1)]
        return np.concatenate(pts)

    def boundary(self):
        """Boundary grid points of a cell relative to its lower-left corner:
        horizontal sides (H grid values, corners included) then vertical sides
        (V grid values, corners excluded).  Returns positions and, per point,
        (lam, ix, iy) with ix, iy the grid offsets in that lambda's units."""
        ns = self.n_s
        out, tags = [], []
        for iy in (0, 1):
            for i in range(ns + 1):
                out.append((i * self.delta, iy * self.L))
                tags.append(("H", i, iy))
        for ix in (0, 1):
            for i in range(1, ns):
                out.append((ix * self.L, i * self.delta))
                tags.append(("V", ix, i))
        return np.array(out), tags


class QRLeastSquares:
    """argmin |A x - b| through a Householder QR of A (the QR-based
    least-squares solution named in eqs. eq_source_point and plwave_QR).
    Each right-hand side is back-substituted (R x = Q^H b); the pseudo-inverse
    is never formed, which keeps the residual small when A is ill-conditioned."""

    def __init__(self, A):
        self.Q, self.R = np.linalg.qr(A, mode="reduced")

    def solve(self, b):
        return solve_triangular(self.R, self.Q.conj().T @ b)


# ---------------------------------------------------------------- kernels
def _green_terms(k, j, h, X, Y, kind):
    """Free-space shifted kernel of eq. (psi_jr_approx), punctured term by term
    (a term whose distance is zero is dropped):
      kind "mono": Phi_j = sum_m w_m (i/4) H0(k R_m)
      kind "dipH": d/dy2 Phi_j = sum_m w_m (ik/4) H1(k R_m) (Y + m h)/R_m
      kind "dipV": d/dy1 Phi_j = sum_m w_m (ik/4) H1(k R_m) X / R_m
    with X = x1 - y1, Y = x2 - y2, R_m = |(X, Y + m h)|."""
    w = greens.shift_weights(j)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.zeros(np.broadcast(X, Y).shape, dtype=np.complex128)
    for m in range(j + 1):
        Ym = Y + m * h
        R = np.hypot(X, Ym)
        ok = R > 1e-9 * max(h, 1e-300) if h > 0 else R > 0
        Rs = np.where(ok, R, 1.0)
        if kind == "mono":
            t = 0.25j * hankel1(0, k * Rs)
        elif kind == "dipH":
            t = 0.25j * k * hankel1(1, k * Rs) * Ym / Rs
        else:
            t = 0.25j * k * hankel1(1, k * Rs) * X / Rs
        out += np.where(ok, w[m] * t, 0.0)
    return out


def _dl0(k, X, Y, fps):
    """Unshifted double-layer kernel per unit dx' (field of one surface true
    source, eq. true_field): (ik/4) H1(kR) (Y - f' X)/R."""
    R = np.hypot(X, Y)
    return 0.25j * k * hankel1(1, k * R) * (Y - fps * X) / R


HYBRID_WINDOW = 8.0


def lattice_table(geom, lam, kind, table="windowed"):
    """Windowed shifted lattice sum of the kernel `kind` (eq. Gq_limit with the
    Bloch phase) on the difference grid of the global grid Pi_lam:
    X = mx * hx, mx = 0..nX-1 (one period), Y = my * hy, my = -(nY-1)..nY-1.
    Returns T[my + nY - 1, mx].  table="hybrid" (Sec. 3.2): the rows that
    greens.hybrid_row_order admits take the spectral series of G~_j instead
    (greens.qper_spectral; no window), the others keep the windowed sums, with
    a window HYBRID_WINDOW times as wide (the spatial series "with a
    sufficiently large value of A" of Sec. 4.2.3)."""
    disc = geom.disc
    k, j, h, d, alpha = disc.k, disc.j, disc.h, disc.d, disc.alpha
    A_len, cA = disc.A * d, disc.c * disc.A * d
    if lam == "H":
        hx, hy, nX, nY = geom.delta, geom.L, geom.n_x * geom.n_s, geom.n_y + 1
    else:
        hx, hy, nX, nY = geom.L, geom.delta, geom.n_x, geom.n_y * geom.n_s + 1 + 2 * geom.n_e
    mx = np.arange(nX)
    my = np.arange(-(nY - 1), nY)
    X = mx[None, :] * hx + 0 * my[:, None]
    Y = my[:, None] * hy + 0 * mx[None, :]
    T = np.zeros(X.shape, dtype=np.complex128)
    spatial = np.ones(len(my), dtype=bool)
    if table == "hybrid":
        for r, yy in enumerate(my * hy):
            nm = greens.hybrid_row_order(k, d, j, h, yy)
            if nm is not None:
                T[r] = greens.qper_spectral(k, alpha, d, j, h, mx * hx, yy, nm, kind)
                spatial[r] = False
    Xs, Ys = X[spatial], Y[spatial]
    if table == "hybrid":
        A_len, cA = HYBRID_WINDOW * A_len, HYBRID_WINDOW * cA
    pmax = int(np.ceil(A_len / d)) + 2
    for p in range(-pmax, pmax + 1):
        Xp = Xs + d * p
        S = greens.window(Xp, cA, A_len)
        if not np.any(S > 0):
            continue
        T[spatial] += np.exp(-1j * alpha * d * p) * S * _green_terms(k, j, h, Xp, Ys, kind)
    return T


# ---------------------------------------------------------------- operator
class AccelOperator:
    """Precomputed tables of Algorithm 2 and the forward map of Algorithm 3."""

    def __init__(self, disc, table="windowed", **geom_kw):
        self.disc = disc
        self.table = table
        g = self.g = Geometry(disc, **geom_kw)
        k = disc.k
        # Equivalent-source least squares, eq. (eq_source_point): A_eq is the same
        # for every cell (relative geometry), so its pseudo-inverse is formed once.
        xc = g.collocation()
        self.pinv = {}
        for lam in ("H", "V"):
            _, _, ys = g.eq_points(lam)
            X = xc[:, None, 0] - ys[None, :, 0]
            Y = xc[:, None, 1] - ys[None, :, 1]
            A = np.concatenate([_green_terms(k, 0, 0.0, X, Y, "mono"),
                                _green_terms(k, 0, 0.0, X, Y, "dip" + lam)], 1)
            self.pinv[lam] = QRLeastSquares(A)
        # per occupied cell: P_q = pinv(A_eq) B_q (B_q: surface true sources -> collocation values)
        self.P = {}
        for c in g.cells:
            idx = g.members[c]
            ox, oy = g.cell_origin(c)
            X = (ox + xc[:, None, 0]) - disc.x[None, idx]
            Y = (oy + xc[:, None, 1]) - disc.f[None, idx]
            B = disc.dx * _dl0(k, X, Y, disc.fp[None, idx])
            self.P[c] = {lam: self.pinv[lam].solve(B) for lam in ("H", "V")}
        # global kernel tables, twisted and Fourier transformed in x
        self.spec = {}
        for lam in ("H", "V"):
            hx = g.delta if lam == "H" else g.L
            Tm = lattice_table(g, lam, "mono", table)
            Td = lattice_table(g, lam, "dip" + lam, table)
            nX = Tm.shape[1]
            tw = np.exp(-1j * disc.alpha * np.arange(nX) * hx)[None, :]
            self.spec[lam] = (np.fft.fft(Tm * tw, axis=1), np.fft.fft(Td * tw, axis=1))
        # plane-wave least squares (eq. plwave_QR), q-independent in cell coordinates
        xb, self.btags = g.boundary()
        ang = 2 * np.pi * np.arange(1, g.n_plw + 1) / g.n_plw
        self.dirs = np.stack([np.sin(ang), np.cos(ang)], 1)
        ctr = np.array([0.5 * g.L, 0.5 * g.L])
        E = np.exp(1j * k * (xb - ctr) @ self.dirs.T)
        self.plw_ls = QRLeastSquares(E)
        self.xb = xb
        self.ctr = ctr
        # near field: band of sources in the three neighbouring columns
        self.near = {}
        for c in g.cells:
            cxq = c % g.n_x
            idx = g.members[c]
            src, shift = [], []
            for ox in range(-g.ring, g.ring + 1):
                col = cxq + ox
                wrap = 0
                if col < 0:
                    col += g.n_x
                    wrap = -1
                elif col >= g.n_x:
                    col -= g.n_x
                    wrap = 1
                s = np.nonzero(g.cx == col)[0]
                src.append(s)
                shift.append(np.full(len(s), wrap))
            src = np.concatenate(src)
            shift = np.concatenate(shift)
            self.near[c] = (idx, src, shift, self._near_block(idx, src, shift))

    # -------------------------------------------------------------- pieces
    def _near_block(self, rows, src, shift):
        """Direct intersecting contributions, eq. (final_correction_0) plus the
        singular part eq. (local_mat) and 1/2 I: the dense operator restricted
        to the source image x_l + p d, p = shift, that lies in the near columns."""
        disc = self.disc
        k, dx = disc.k, disc.dx
        X = disc.x[rows, None] - (disc.x[None, src] + shift[None, :] * disc.d)
        Y = disc.f[rows, None] - disc.f[None, src]
        FPS = np.broadcast_to(disc.fp[None, src], X.shape)
        diag = (rows[:, None] == src[None, :]) & (shift[None, :] == 0)
        M = np.zeros(X.shape, dtype=np.complex128)
        off = ~diag
        K = np.zeros(X.shape, dtype=np.complex128)
        K[off] = greens.dlayer_kernel(k, disc.j, disc.h, X[off], Y[off], FPS[off])
        Sf = greens.window(np.hypot(X, Y), disc.gamma, disc.a)
        M += dx * (1.0 - Sf) * K * off
        sing = off & (Sf > 0)
        if np.any(sing):
            Ks = greens.mk_log_coefficient(k, X[sing], Y[sing], FPS[sing])
            Kr = K[sing] - Ks * greens.mk_log_factor(X[sing], disc.a)
            Rw = greens.log_weights(disc.n_a, dx, np.rint(-X[sing] / dx))
            M[sing] += Sf[sing] * (Rw * Ks + dx * Kr)
        rr, cc = np.nonzero(diag)
        Krd = greens.mk_smooth_diagonal(k, disc.j, disc.h, disc.fp[rows[rr]], disc.fpp[rows[rr]])
        M[rr, cc] += dx * Krd + 0.5
        phase = np.exp(1j * disc.alpha * shift * disc.d)[None, :]
        return M * phase

    def eq_sources(self, mu):
        """EqSources: (xi, zeta)^{q,lam} = P_q^lam mu|_q for every occupied cell."""
        return {c: {lam: self.P[c][lam] @ mu[self.g.members[c]] for lam in ("H", "V")} for c in self.g.cells}

    def global_merge(self, dens):
        """GlobalEqSMerge, eq. (sum_eqsources): add the cell densities at shared
        points of the periodic grids; points beyond the period are wrapped with
        exp(-/+ i alpha d) (densities are alpha-quasi-periodic, Remark
        eq_source_quasiper)."""
        g, disc = self.g, self.disc
        grids = {}
        nXH, nYH = g.n_x * g.n_s, g.n_y + 1
        nXV, nYV = g.n_x, g.n_y * g.n_s + 1 + 2 * g.n_e
        for lam, (nX, nY) in (("H", (nXH, nYH)), ("V", (nXV, nYV))):
            xi = np.zeros((nY, nX), dtype=np.complex128)
            ze = np.zeros((nY, nX), dtype=np.complex128)
            ix, iy, _ = g.eq_points(lam)
            n = len(ix)
            for c, dd in dens.items():
                cxq, cyq = c % g.n_x, c // g.n_x
                if lam == "H":
                    gx = cxq * g.n_s + ix
                    gy = cyq + iy
                else:
                    gx = cxq + ix
                    gy = cyq * g.n_s + iy + g.n_e
                wrap = np.floor_divide(gx, nX)
                gx = gx - wrap * nX
                ph = np.exp(-1j * disc.alpha * disc.d * wrap)
                np.add.at(xi, (gy, gx), ph * dd[lam][:n])
                np.add.at(ze, (gy, gx), ph * dd[lam][n:])
            grids[lam] = (xi, ze)
        return grids

    def global_fft(self, grids):
        """GlobalFFT, eq. (large_convolution_per_grid): phi^all on each grid."""
        g, disc = self.g, self.disc
        out = {}
        for lam in ("H", "V"):
            xi, ze = grids[lam]
            nY, nX = xi.shape
            hx = g.delta if lam == "H" else g.L
            tw = np.exp(-1j * disc.alpha * np.arange(nX) * hx)[None, :]
            Fx = np.fft.fft(xi * tw, axis=1)
            Fz = np.fft.fft(ze * tw, axis=1)
            Km, Kd = self.spec[lam]
            phi = np.zeros((nY, nX), dtype=np.complex128)
            for t in range(nY):
                for tp in range(nY):
                    r = t - tp + nY - 1
                    phi[t] += Km[r] * Fx[tp] + Kd[r] * Fz[tp]
            out[lam] = np.fft.ifft(phi, axis=1) / tw
        return out

    def boundary_values(self, c, phi_all, dens):
        """LocalEqSMerge + LocalFFT + LocalSubtract + Combine-lambda: the
        non-intersecting field on the boundary grid points of cell c
        (eqs. small_convolution, psi_na_sum, combine_psi_pna)."""
        g, disc = self.g, self.disc
        k, j, h = disc.k, disc.j, disc.h
        cxq, cyq = c % g.n_x, c // g.n_x
        ox, oy = g.cell_origin(c)
        vals = np.zeros(len(self.btags), dtype=np.complex128)
        for b, (lam, ix, iy) in enumerate(self.btags):
            if lam == "H":
                gx, gy = cxq * g.n_s + ix, cyq + iy
                nX = g.n_x * g.n_s
            else:
                gx, gy = cxq + ix, cyq * g.n_s + iy + g.n_e
                nX = g.n_x
            wrap = gx // nX
            vals[b] = phi_all[lam][gy, gx - wrap * nX] * np.exp(1j * disc.alpha * disc.d * wrap)
        # subtract the equivalent sources of every cell in the three columns
        xb = self.xb + np.array([ox, oy])
        for b, (lam, _, _) in enumerate(self.btags):
            _, _, ys = g.eq_points(lam)
            n = len(ys)
            for dxc in range(-g.ring, g.ring + 1):
                for r_y in range(g.n_y):
                    col = cxq + dxc
                    wrap = 0
                    if col < 0:
                        col, wrap = col + g.n_x, -1
                    elif col >= g.n_x:
                        col, wrap = col - g.n_x, 1
                    r = r_y * g.n_x + col
                    if r not in dens:
                        continue
                    rx0, ry0 = g.cell_origin(r)
                    rx0 += wrap * disc.d
                    X = xb[b, 0] - (rx0 + ys[:, 0])
                    Y = xb[b, 1] - (ry0 + ys[:, 1])
                    ph = np.exp(1j * disc.alpha * disc.d * wrap)
                    v = dens[r][lam]
                    vals[b] -= ph * (np.sum(_green_terms(k, j, h, X, Y, "mono") * v[:n])
                                     + np.sum(_green_terms(k, j, h, X, Y, "dip" + lam) * v[n:]))
        return vals

    def matvec(self, mu, return_parts=False):
        disc, g = self.disc, self.g
        y = np.zeros(disc.N, dtype=np.complex128)
        dens = self.eq_sources(mu)
        grids = self.global_merge(dens)
        phi_all = self.global_fft(grids)
        far = np.zeros(disc.N, dtype=np.complex128)
        for c in g.cells:
            rows, src, shift, Mq = self.near[c]
            y[rows] += Mq @ mu[src]                                  # Intersecting, EvalSingular, 1/2 I
            b = self.boundary_values(c, phi_all, dens)
            w = self.plw_ls.solve(b)                                  # PlaneWaveWeights
            ox, oy = g.cell_origin(c)
            pts = np.stack([disc.x[rows] - ox, disc.f[rows] - oy], 1) - self.ctr
            far[rows] = np.exp(1j * disc.k * pts @ self.dirs.T) @ w   # NonIntersecting
        y += far
        for n in disc.U_eta:                                          # EvalModes
            an = rayleigh.alpha_n(disc.alpha, disc.d, n)
            bn = greens.beta_of(disc.k, np.array([an]))[0]
            s = np.sum(np.exp(-1j * an * disc.x - 1j * bn * disc.f) * disc.J * disc.dx * mu)
            y += np.exp(1j * an * disc.x + 1j * bn * disc.f) * s
        if return_parts:
            return y, dict(dens=dens, grids=grids, phi_all=phi_all, far=far)
        return y
