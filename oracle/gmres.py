"""Unrestarted GMRES (oracle; test infrastructure).

The paper solves eq. (discrete_eq) iteratively with GMRES (Saad-Schultz);
this is the textbook algorithm: Arnoldi with modified Gram-Schmidt, Givens
rotations on the Hessenberg matrix, x0 = 0, stop when the residual norm
estimate falls below tol * ||b||.
"""
import numpy as np


def gmres(apply, b, tol=1e-10, max_iter=500):
    """Return (x, iterations, relative residual estimate)."""
    n = b.shape[0]
    beta0 = np.linalg.norm(b)
    if beta0 == 0.0:
        return np.zeros_like(b), 0, 0.0
    m = max_iter
    V = np.zeros((m + 1, n), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    cs = np.zeros(m, dtype=np.complex128)
    sn = np.zeros(m, dtype=np.complex128)
    g = np.zeros(m + 1, dtype=np.complex128)
    g[0] = beta0
    V[0] = b / beta0
    it = 0
    res = 1.0
    for it in range(1, m + 1):
        jcol = it - 1
        w = apply(V[jcol])
        for i in range(it):
            H[i, jcol] = np.vdot(V[i], w)
            w = w - H[i, jcol] * V[i]
        H[it, jcol] = np.linalg.norm(w)
        if H[it, jcol] != 0:
            V[it] = w / H[it, jcol]
        # apply the previous rotations G_i = [[conj(c), conj(s)], [-s, c]]
        for i in range(jcol):
            u, v = H[i, jcol], H[i + 1, jcol]
            H[i, jcol] = np.conj(cs[i]) * u + np.conj(sn[i]) * v
            H[i + 1, jcol] = -sn[i] * u + cs[i] * v
        a, bb = H[jcol, jcol], H[jcol + 1, jcol]
        r = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
        cs[jcol] = a / r if r != 0 else 1.0
        sn[jcol] = bb / r if r != 0 else 0.0
        H[jcol, jcol] = r
        H[jcol + 1, jcol] = 0.0
        g[jcol + 1] = -sn[jcol] * g[jcol]
        g[jcol] = np.conj(cs[jcol]) * g[jcol]
        res = abs(g[jcol + 1]) / beta0
        if res < tol:
            break
    y = np.linalg.solve(np.triu(H[:it, :it]), g[:it])
    x = V[:it].T @ y
    return x, it, res
