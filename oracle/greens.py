"""Green functions, windows and quadrature weights (oracle; test infrastructure).

Everything here is plain NumPy/SciPy in FP64 and follows the paper's
definitions directly:

* free-space Green function G = (i/4) H0^(1)(k r)                 eq. (free_space)
* multipolar ("shifted") Green function
      G_j(X,Y) = sum_m (-1)^m C(j,m) G(X, Y + m h)             eq. (shifted_green_function)
* the smooth windows S_{gamma,a}                                  eq. (S_def)
* the windowed spatial lattice sum G~^{q,A}_j                     eq. (Gq_limit)
  with the Bloch phase exp(-i alpha d p) that eq. (Gq_limit) omits and
  eq. (shifted_periodic_green_function) carries
* the spectral (Rayleigh) series of G~_j                          eq. (shifted_quasi_per_rayleigh)
  and its form valid at Wood anomalies                           eq. (betan_taylor), Sec. 3.2
* the double-layer kernel, the Martensen-Kussmaul split K_s, K_r and the
  Fourier-based log-quadrature weights R                          Sec. 4.2.1, eqs. (descomp)-(local_mat)

Kernel normalisation.  With the unnormalised upward normal n' = (-f'(x'), 1)
one has nu(x') ds' = n' dx', so the double-layer integrand per unit dx' is
    K_dl(X, Y; f'(x')) = f'(x') dG_j/dX - dG_j/dY
                       = sum_m (-1)^m C(j,m) (i k/4) H1(k R_m) (Y + m h - f'(x') X) / R_m,
with X = x - x', Y = f(x) - f(x'), R_m = |(X, Y + m h)|.  Eq. (K_def) defines
the derivative with respect to the source point; the upward normal is the one
for which eq. (eq_per_doublelayer) carries +1/2.
"""
from math import comb

import numpy as np
from scipy.special import hankel1, j1


def shift_weights(j):
    """(-1)^m C(j, m), m = 0..j (eq. shifted_green_function)."""
    return np.array([(-1) ** m * comb(j, m) for m in range(j + 1)], dtype=np.float64)


def window(x, gamma, a):
    """S_{gamma,a}(x) of eq. (S_def): 1 on |x| <= gamma, exp(2 e^{-1/u}/(u-1))
    with u = (|x|-gamma)/(a-gamma) on gamma < |x| < a, 0 on |x| >= a."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros(x.shape)
    out[x <= gamma] = 1.0
    mid = (x > gamma) & (x < a)
    u = (x[mid] - gamma) / (a - gamma)
    out[mid] = np.exp(2.0 * np.exp(-1.0 / u) / (u - 1.0))
    return out


def green(k, X, Y):
    """G(X,Y) = (i/4) H0^(1)(k sqrt(X^2+Y^2)), eq. (free_space)."""
    return 0.25j * hankel1(0, k * np.hypot(X, Y))


def green_shifted(k, j, h, X, Y):
    """G_j(X,Y), eq. (shifted_green_function)."""
    w = shift_weights(j)
    return sum(w[m] * green(k, X, Y + m * h) for m in range(j + 1))


def dlayer_kernel(k, j, h, X, Y, fps):
    """Double-layer kernel per unit dx' (see module docstring).

    X = x - x', Y = f(x) - f(x'), fps = f'(x').  Undefined at X = Y = 0
    (the m = 0 term is singular there); callers exclude that point.
    """
    w = shift_weights(j)
    out = np.zeros(np.broadcast(X, Y, fps).shape, dtype=np.complex128)
    for m in range(j + 1):
        Ym = Y + m * h
        R = np.hypot(X, Ym)
        out += w[m] * (0.25j * k) * hankel1(1, k * R) * (Ym - fps * X) / R
    return out


def mk_log_coefficient(k, X, Y, fps):
    """K_s of eq. (ks_def), read as (k/4pi) [f'(x')(x-x') - (f(x)-f(x'))] J1(kR)/R.

    The printed formula has f(x') for f'(x') and the opposite sign on the
    height difference; with those slips the bracket would not vanish on a
    straight line, whereas the logarithmic part of H1 (through
    Y1(z) ~ (2/pi) J1(z) ln(z/2)) carries exactly this coefficient.
    K_s vanishes at X = Y = 0.
    """
    R = np.hypot(X, Y)
    Rs = np.where(R == 0.0, 1.0, R)
    val = (k / (4.0 * np.pi)) * (fps * X - Y) * j1(k * Rs) / Rs
    return np.where(R == 0.0, 0.0, val)


def mk_log_factor(X, a):
    """ln(4 sin^2(pi X / a)), the periodic logarithm of eq. (descomp)."""
    return np.log(4.0 * np.sin(np.pi * np.asarray(X) / a) ** 2)


def mk_smooth_diagonal(k, j, h, fp, fpp):
    """K_r(x,x): the limit of K_r of eq. (kr_def) as x' -> x.

    The m = 0 term tends to f''/(4 pi (1+f'^2)) (the curvature term of the
    double layer); each shifted term m >= 1 is evaluated at X = 0, Y = 0,
    where R_m = m h and the geometric factor equals 1.
    """
    w = shift_weights(j)
    val = fpp / (4.0 * np.pi * (1.0 + fp * fp)) + 0j
    for m in range(1, j + 1):
        val = val + w[m] * (0.25j * k) * hankel1(1, k * m * h)
    return val


def log_weights(n_a, dx, m):
    """Fourier-based weights R_m for int_{-a}^{a} ln(4 sin^2(pi t/a)) g(t) dt
    with a = n_a dx and nodes t = m dx (eq. local_mat).

    The paper obtains them by following Bruno-Delourme Sec. 5.2; that
    derivation is not reproduced in the paper, so it is done here from the
    same principle: integrate exactly the trigonometric interpolant of g of
    period 2a through the 2 n_a nodes, using
        int_{-a}^{a} ln(4 sin^2(pi t/a)) exp(i pi q t / a) dt
            = -4a/|q|  (q even, q != 0),   0  (q odd or q = 0),
    which follows from ln(4 sin^2(s/2)) = -2 sum_{n>=1} cos(n s)/n.  This
    gives R_m = -2 dx sum_{s=1}^{floor(n_a/2)} w_s cos(2 pi s m / n_a) / s,
    w_s = 1/2 for 2s = n_a (the Nyquist term) and 1 otherwise.
    """
    m = np.asarray(m, dtype=np.float64)
    out = np.zeros(m.shape)
    for s in range(1, n_a // 2 + 1):
        ws = 0.5 if 2 * s == n_a else 1.0
        out += ws * np.cos(2.0 * np.pi * s * m / n_a) / s
    return -2.0 * dx * out


def lattice_sum_windowed(k, alpha, d, j, h, A_len, c, X, Y, kernel="G", fps=0.0):
    """Windowed spatial lattice sum, eq. (Gq_limit) with the Bloch phase:
        sum_p exp(-i alpha d p) S_{cA,A}(X + d p) K(X + d p, Y),
    K = G_j ("G") or the double-layer kernel ("dl", with source slope fps).
    A_len is the window half-width in length units.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    pmax = int(np.ceil(A_len / d)) + 1
    out = np.zeros(np.broadcast(X, Y).shape, dtype=np.complex128)
    for p in range(-pmax, pmax + 1):
        Xp = X + d * p
        S = window(Xp, c * A_len, A_len)
        if not np.any(S > 0):
            continue
        if kernel == "G":
            K = green_shifted(k, j, h, Xp, Y)
        else:
            K = dlayer_kernel(k, j, h, Xp, Y, fps)
        out += np.exp(-1j * alpha * d * p) * S * K
    return out


def beta_of(k, alpha_n):
    """beta_n of eq. (alpha_beta_def): sqrt(k^2-alpha_n^2) if positive,
    i sqrt(alpha_n^2-k^2) otherwise (positive branches)."""
    disc = k * k - np.asarray(alpha_n, dtype=np.float64) ** 2
    return np.where(disc >= 0, np.sqrt(np.abs(disc)) + 0j, 1j * np.sqrt(np.abs(disc)))


def lattice_sum_spectral(k, alpha, d, j, h, X, Y, nmax, kernel="G", fps=0.0):
    """Spectral series of G~_j, eq. (shifted_quasi_per_rayleigh), truncated to
    |n| <= nmax; valid (exponentially convergent) where every |Y + m h| is
    bounded away from 0.  kernel="dl" returns f' dG/dX - dG/dY of the same
    series, term by term.  Not for exact Wood anomalies (beta_n = 0)."""
    w = shift_weights(j)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.zeros(np.broadcast(X, Y).shape, dtype=np.complex128)
    for n in range(-nmax, nmax + 1):
        an = alpha + 2.0 * np.pi * n / d
        bn = beta_of(k, an)
        ex = np.exp(1j * an * X)
        for m in range(j + 1):
            Ym = Y + m * h
            e = np.exp(1j * bn * np.abs(Ym))
            if kernel == "G":
                term = e
            else:
                term = (fps * 1j * an - 1j * bn * np.sign(Ym)) * e
            out += w[m] * (1j / (2.0 * d * bn)) * ex * term
    return out


# ---------------------------------------------------------------- Sec. 3.2: spectral series at Wood anomalies
def _q_pow(beta, h, j):
    """(1 - e^{i beta h})^j / beta for j >= 1 (beta complex, scalar): directly
    for |beta| >= 0.5, else with (1 - e^{i beta h}) / beta summed as its Taylor
    series -i h sum_{n>=0} (i beta h)^n / (n+1)!."""
    z = 1j * beta * h
    if abs(beta) >= 0.5:
        return (1.0 - np.exp(z)) ** j / beta
    q, term, n = 0j, 1.0 + 0j, 0
    while True:
        add = term / _fact(n + 1)
        q += add
        if abs(add) < 1e-20 * max(abs(q), 1e-300) or n > 60:
            break
        n += 1
        term *= z
    q *= -1j * h  # (1 - e^{i beta h}) / beta
    return q ** j * beta ** (j - 1)


def _q_odd(beta, t):
    """(e^{i beta t} - e^{-i beta t}) / beta = 2i sin(beta t) / beta: directly
    for |beta| >= 0.5, else as 2i sum_{n>=0} (-1)^n beta^{2n} t^{2n+1} / (2n+1)!."""
    if abs(beta) >= 0.5:
        return (np.exp(1j * beta * t) - np.exp(-1j * beta * t)) / beta
    s, n = 0j, 0
    b2 = beta * beta
    term = t + 0j
    while True:
        add = term / _fact(2 * n + 1)
        s += add
        if abs(add) < 1e-20 * max(abs(s), 1e-300) or n > 60:
            break
        n += 1
        term *= -b2 * t * t
    return 2j * s


def _fact(n):
    out = 1.0
    for i in range(2, n + 1):
        out *= i
    return out


def qper_spectral(k, alpha, d, j, h, X, Y, nmax, kind="mono"):
    """G~_j (eq. shifted_periodic_green_function) from its spectral series, eq.
    (shifted_quasi_per_rayleigh), summed over |n| <= nmax, for points whose
    height Y keeps away from every shifted pole row Y = -m h (then the terms
    decay like exp(-|beta_n| min_m |Y + m h|), eq. spectral_exp_estimate).  The
    beta_n-quotient of each term is taken in the form of eq. (betan_taylor),
        sum_m w_m e^{i beta |Y+mh|} / beta
          = e^{i beta Y} (1 - e^{i beta h})^j / beta
            - sum_{m: Y+mh < 0} w_m (e^{i beta (Y+mh)} - e^{-i beta (Y+mh)}) / beta,
    with both quotients summed as Taylor series, for |beta_n| < 0.5, so the
    series also holds at Wood anomalies (beta_n = 0; needs j >= 1); the other
    terms take the quotient as printed.
    kind: "mono" G~_j; "dipH" -dG~_j/dY (derivative in the source height);
    "dipV" -dG~_j/dX (in the source abscissa).  X: array, Y: scalar."""
    assert j >= 1
    w = shift_weights(j)
    X = np.asarray(X, dtype=np.float64)
    Y = float(Y)
    out = np.zeros(X.shape, dtype=np.complex128)
    for n in range(-nmax, nmax + 1):
        an = alpha + 2.0 * np.pi * n / d
        g = (k - an) * (k + an)
        bn = np.sqrt(g) + 0j if g >= 0 else 1j * np.sqrt(-g)
        ts = Y + h * np.arange(j + 1)
        if kind == "dipH":
            coef = np.sum(w * np.sign(ts) * np.exp(1j * bn * np.abs(ts))) / (2.0 * d)
        else:
            if abs(bn) >= 0.5:  # the plain quotient (the closed form would cancel for evanescent terms)
                q = np.sum(w * np.exp(1j * bn * np.abs(ts))) / bn
            else:
                q = np.exp(1j * bn * Y) * _q_pow(bn, h, j)
                for m in range(j + 1):
                    if ts[m] < 0:
                        q -= w[m] * _q_odd(bn, ts[m])
            coef = (1j if kind == "mono" else an) * q / (2.0 * d)
        out += coef * np.exp(1j * an * X)
    return out


def hybrid_row_order(k, d, j, h, Y):
    """The hybrid tables' choice for a row at height Y (Sec. 3.2): the
    truncation order of its spectral series, or None when the row keeps the
    windowed sums.  delta = min_m |Y + m h|; the terms fall below e^{-42}
    where |beta_n| delta > 42, i.e. beyond |alpha_n| = sqrt((42/delta)^2 + k^2),
    and |alpha| < k; rows needing more than 40000 orders, or on a pole row,
    keep the windowed sums."""
    delta = min(abs(Y + m * h) for m in range(j + 1))
    if not delta > 0:
        return None
    nm = int(np.ceil((np.sqrt((42.0 / delta) ** 2 + k * k) + k) * d / (2.0 * np.pi))) + 2
    return nm if nm <= 40000 else None
