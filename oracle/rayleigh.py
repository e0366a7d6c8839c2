"""Rayleigh wavenumbers, completion set, Rayleigh coefficients, efficiencies
(oracle; test infrastructure).

Sec. 2: alpha_n = alpha + 2 pi n / d, beta_n per eq. (alpha_beta_def);
propagating set U = {n : k^2 - alpha_n^2 > 0}; efficiencies
e_n = (beta_n / beta) |B_n|^2 and energy-balance error eq. (energy_error).
Sec. 3.1: completion function M^eta and its index set U^eta, eq. (M_eta).
"""
import numpy as np

from .greens import beta_of


def alpha_n(alpha, d, n):
    return alpha + 2.0 * np.pi * np.asarray(n, dtype=np.float64) / d


def propagating_orders(k, alpha, d):
    """U: integers n with k^2 - alpha_n^2 > 0."""
    nlo = int(np.floor((-k - alpha) * d / (2 * np.pi))) - 1
    nhi = int(np.ceil((k - alpha) * d / (2 * np.pi))) + 1
    n = np.arange(nlo, nhi + 1)
    an = alpha_n(alpha, d, n)
    return n[k * k - an * an > 0]


def shift_factor_abs(k, an, h, j):
    """|1 - exp(i beta_n h)|^j."""
    bn = beta_of(k, an)
    return np.abs(1.0 - np.exp(1j * bn * h)) ** j


def completion_set(k, alpha, d, h, j, eta):
    """U^eta of eq. (M_eta), read as {n : |1 - exp(i beta_n h)|^j < eta}.

    As printed, the test |(1 - e^{i beta_n h})^j / beta_n| < eta holds for
    every evanescent order with |n| large enough (the quotient decays like
    d / (2 pi |n|)), which would make U^eta infinite.  The quantity that
    matters is the size of the factor the shift puts on mode n: on a flat
    surface (1/2 I + D~) maps exp(i alpha_n x) to (1/2)(1 - e^{i beta_n h})^j
    times itself, so modes whose factor is below eta are the ones to
    complete.  For j = 0 the set is empty.
    """
    if j == 0:
        return np.zeros(0, dtype=np.int64)
    # evanescent orders with kappa h beyond this bound have factor > eta
    t = eta ** (1.0 / j)
    kappa_max = -np.log(1.0 - min(t, 0.999999)) / h + 1.0
    K = np.sqrt(k * k + kappa_max * kappa_max)
    nlo = int(np.floor((-K - alpha) * d / (2 * np.pi))) - 1
    nhi = int(np.ceil((K - alpha) * d / (2 * np.pi))) + 1
    n = np.arange(nlo, nhi + 1)
    fac = shift_factor_abs(k, alpha_n(alpha, d, n), h, j)
    return n[fac < eta]


def shift_quotient(k, an, h, j):
    """(1 - exp(i beta_n h))^j / beta_n, with its beta_n -> 0 limit.

    Uses 1 - e^{iz} = -2i sin(z/2) e^{iz/2} so that small beta_n loses no
    digits.
    """
    bn = beta_of(k, an)
    z = bn * h
    out = np.empty(bn.shape, dtype=np.complex128)
    zero = bn == 0
    nz = ~zero
    out[nz] = ((-2j) ** j * np.sin(z[nz] / 2) ** j * np.exp(0.5j * j * z[nz])) / bn[nz]
    if j >= 2:
        out[zero] = 0.0
    elif j == 1:
        out[zero] = -1j * h
    else:
        out[zero] = np.inf
    return out


def rayleigh_coefficients(disc, mu, orders):
    """B_n for y > max f.

    The paper does not print this formula; it follows from inserting the
    spectral series eq. (shifted_periodic_green_function_spectral) (valid for
    Y > 0) and M^eta of eq. (M_eta) into the representation
    eq. (eq:int_eq_dirichlet), and applying the trapezoidal rule:
      B_n = dx sum_l [ -(alpha_n f'_l - beta_n) (1 - e^{i beta_n h})^j / (2 d beta_n)
                       + 1[n in U^eta] J_l ] exp(-i alpha_n x_l - i beta_n f_l) mu_l,
    with J_l = sqrt(1 + f'_l^2).
    """
    orders = np.asarray(orders)
    an = alpha_n(disc.alpha, disc.d, orders)
    bn = beta_of(disc.k, an)
    Q = shift_quotient(disc.k, an, disc.h, disc.j)
    inU = np.isin(orders, disc.U_eta)
    B = np.zeros(len(orders), dtype=np.complex128)
    for t in range(len(orders)):
        dl = -(an[t] * disc.fp - bn[t]) * Q[t] / (2.0 * disc.d)
        if inU[t]:
            dl = dl + disc.J
        B[t] = disc.dx * np.sum(dl * np.exp(-1j * an[t] * disc.x - 1j * bn[t] * disc.f) * mu)
    return B


def efficiencies(disc, mu):
    """Return (orders n in U, e_n, energy-balance error eps)."""
    orders = propagating_orders(disc.k, disc.alpha, disc.d)
    B = rayleigh_coefficients(disc, mu, orders)
    bn = beta_of(disc.k, alpha_n(disc.alpha, disc.d, orders)).real
    e = bn / disc.beta * np.abs(B) ** 2
    return orders, e, 1.0 - float(np.sum(e))
