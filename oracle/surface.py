"""Surface profile and quadrature nodes (oracle; test infrastructure).

Sec. 4.2 (discretisation): equispaced nodes x_l = l dx with dx = d/N.  The
paper numbers nodes 1..N with x_N = d; this implementation stores the same
node set shifted by one period on the first node, x_l = l dx for l = 0..N-1,
which by alpha-quasi-periodicity of the density (eq. quasiper_disc) only
re-labels one unknown.

The profile is a real trigonometric polynomial
    f(x) = a_0 + sum_m a_m cos(2 pi m x/d) + b_m sin(2 pi m x/d),
evaluated exactly together with f' and f''.
"""
import numpy as np


def nodes(d, N):
    return np.arange(N, dtype=np.float64) * (d / N)


def profile(a_coef, b_coef, d, x):
    """Return f, f', f'' at the points x (float64 arrays)."""
    a = np.asarray(a_coef, dtype=np.float64)
    b = np.zeros_like(a)
    bb = np.asarray(b_coef, dtype=np.float64)
    b[: len(bb)] = bb[: len(a)]
    x = np.asarray(x, dtype=np.float64)
    f = np.full(x.shape, a[0])
    fp = np.zeros(x.shape)
    fpp = np.zeros(x.shape)
    for m in range(1, len(a)):
        w = 2.0 * np.pi * m / d
        c = np.cos(w * x)
        s = np.sin(w * x)
        f += a[m] * c + b[m] * s
        fp += w * (-a[m] * s + b[m] * c)
        fpp += -w * w * (a[m] * c + b[m] * s)
    return f, fp, fpp
