"""Dense direct Nystrom operator (1/2 I + D^dx) (oracle; test infrastructure).

Sec. 4.3, eqs. (D_deltax)-(discrete_eq): D^dx = D~_sing^dx + D~_reg^dx + D_M^dx.

* D~_reg^{A,dx} is the windowed trapezoidal rule of eq. (DAdx_def): every
  source node x_l of the real line (the images of the N nodes of one period,
  with mu_{k+pN} = mu_k e^{i alpha p d}, eq. quasiper_disc) contributes
      dx S_{cA,A}(x_i - x_l) (1 - S^f_{gamma,a}(x_i, x_l)) K_dl mu_l.
  The window S^f uses the two-dimensional distance, as in eqs. (dsing_def)
  and (DAdx_def), so that D~_sing + D~_reg reproduce D~ exactly.
* D~_sing^dx is eq. (local_mat) with W = dx (trapezoid) and the Fourier-based
  log weights R of greens.log_weights:
      S^f (R_{l-i} K_s + dx K_r) mu_l,   K_r = K_dl - K_s ln(4 sin^2(pi X/a)),
  and K_r(x,x) from greens.mk_smooth_diagonal on the diagonal.
* D_M^dx is the trapezoidal rule for eq. (per_doublelayer_DM) with the kernel
  M^eta of eq. (M_eta):
      sum_{n in U^eta} exp(i alpha_n (x_i - x_l) + i beta_n (f_i - f_l)) J_l dx.
  (Eq. (D_M_deltax) as printed drops exp(i beta_n f(x_i)) and exp(-i alpha_n
  x_l) and flips the sign of beta_n f(x_l); the kernel of eq. (M_eta) is used
  as defined.)
"""
import numpy as np

from . import greens, rayleigh
from .surface import nodes, profile


class Discretization:
    """Nodes, profile samples and all scalar parameters of one problem.

    Built from a workloads.Workload (or anything with the same attributes).
    """

    def __init__(self, wl, N=None, n_a=None):
        self.N = int(N if N is not None else wl.N)
        self.d = float(wl.d)
        self.k = float(wl.k)
        self.alpha = float(wl.alpha)
        self.beta = float(wl.beta)
        self.j = int(wl.j)
        self.h = float(wl.h)
        self.A = float(wl.A)
        self.c = float(wl.c)
        self.eta = float(wl.eta)
        self.dx = self.d / self.N
        if n_a is None:
            n_a = wl.n_a if wl.n_a else None
        if n_a is None:
            # a = n_a dx slightly below the cell side (a < L, a < d)
            n_a = max(8, int(np.floor(0.8 * min(wl.L, self.d) / self.dx)))
        self.n_a = int(n_a)
        self.a = self.n_a * self.dx
        self.gamma = float(wl.gamma_frac) * self.a
        self.x = nodes(self.d, self.N)
        self.f, self.fp, self.fpp = profile(wl.a_coef, wl.b_coef, self.d, self.x)
        self.J = np.sqrt(1.0 + self.fp ** 2)
        self.U_eta = rayleigh.completion_set(self.k, self.alpha, self.d, self.h, self.j, self.eta)


def rhs(disc):
    """b_i = -u^inc(x_i, f(x_i)) = -exp(i (alpha x_i - beta f_i)), eq. (fist_eq)."""
    return -np.exp(1j * (disc.alpha * disc.x - disc.beta * disc.f))


def operator_rows(disc, rows):
    """Rows `rows` of the N x N matrix of (1/2 I + D^dx)."""
    rows = np.atleast_1d(np.asarray(rows, dtype=np.int64))
    N, d, dx, k = disc.N, disc.d, disc.dx, disc.k
    A_len = disc.A * d
    cols = np.arange(N)
    X0 = disc.x[rows, None] - disc.x[None, :]
    Y = disc.f[rows, None] - disc.f[None, :]
    FPS = np.broadcast_to(disc.fp[None, :], X0.shape)
    diag = rows[:, None] == cols[None, :]
    M = np.zeros(X0.shape, dtype=np.complex128)
    pmax = int(np.ceil(disc.A)) + 1
    for p in range(-pmax, pmax + 1):
        # source node x_l = x_k + p d, mu_l = mu_k exp(i alpha p d)
        Xp = X0 - p * d
        SA = greens.window(Xp, disc.c * A_len, A_len)
        act = SA > 0
        if p == 0:
            act &= ~diag
        if not np.any(act):
            continue
        Sf = greens.window(np.hypot(Xp, Y), disc.gamma, disc.a)
        K = np.zeros(X0.shape, dtype=np.complex128)
        K[act] = greens.dlayer_kernel(k, disc.j, disc.h, Xp[act], Y[act], FPS[act])
        phase = np.exp(1j * disc.alpha * p * d)
        # regular part, eq. (DAdx_def)
        M += phase * dx * SA * (1.0 - Sf) * K
        # singular part, eq. (local_mat), off-diagonal pairs with S^f > 0
        sing = act & (Sf > 0)
        if np.any(sing):
            Xs, Ys = Xp[sing], Y[sing]
            Ks = greens.mk_log_coefficient(k, Xs, Ys, FPS[sing])
            Kr = K[sing] - Ks * greens.mk_log_factor(Xs, disc.a)
            midx = np.rint(-Xs / dx)          # l - i for the source l
            Rw = greens.log_weights(disc.n_a, dx, midx)
            M[sing] += phase * Sf[sing] * (Rw * Ks + dx * Kr)
    # diagonal: S^f = 1, K_s(x,x) = 0, so D~_sing contributes dx K_r(x,x)
    Krd = greens.mk_smooth_diagonal(k, disc.j, disc.h, disc.fp[rows], disc.fpp[rows])
    M[np.arange(len(rows)), rows] += dx * Krd + 0.5
    # completion modes D_M
    for n in disc.U_eta:
        an = rayleigh.alpha_n(disc.alpha, d, n)
        bn = greens.beta_of(k, an)
        M += np.exp(1j * an * X0 + 1j * bn * Y) * (disc.J * dx)[None, :]
    return M


def operator_matrix(disc, block=64):
    """The full N x N matrix, assembled in row blocks."""
    out = np.empty((disc.N, disc.N), dtype=np.complex128)
    for s in range(0, disc.N, block):
        r = np.arange(s, min(disc.N, s + block))
        out[r] = operator_rows(disc, r)
    return out


def matvec_rows(disc, mu, rows):
    """((1/2 I + D^dx) mu)[rows], assembling only those rows."""
    return operator_rows(disc, rows) @ mu
