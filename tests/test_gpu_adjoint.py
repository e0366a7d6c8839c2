"""Adjoint gradients (dense mode) through the C ABI: the conjugate-transpose
map against the oracle's matrix, the adjoint solve, the objective and its
adjoint right-hand side against the oracle's Rayleigh coefficients, and the
shape gradient of an efficiency objective with respect to the profile's
Fourier coefficients against finite differences (central, step 1e-6, and
Richardson-extrapolated) of the oracle's objective (dense LU + efficiencies)
and of the library's own solves; the torch.autograd.Function gives the same
gradient.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, rayleigh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def solver(torch):
    import paper_1707_04950_amd as lib
    s = lib.Solver(0)
    yield s
    s.close()


def _surface_kw(wl, disc):
    return dict(d=wl.d, k=wl.k, alpha=wl.alpha, j=wl.j, A=wl.A, N=disc.N, h=wl.h, c=wl.c, n_a=disc.n_a,
                gamma_frac=wl.gamma_frac, eta=wl.eta, L=wl.L)


def _set(solver, wl, a=None, b=None, adjoint=0):
    import paper_1707_04950_amd as lib
    disc = dense.Discretization(wl)
    solver.set_surface(np.asarray(wl.a_coef if a is None else a), np.asarray(wl.b_coef if b is None else b),
                       mode=lib.MODE_DENSE, adjoint=adjoint, **_surface_kw(wl, disc))
    return disc


def _case():
    # the sinusoid with two more modes, so that every coefficient below is active
    wl = W.config_dense_sinusoid(256)
    return wl.with_(a_coef=(0.0, 0.3125, 0.04), b_coef=(0.0, 0.05, -0.03))


def test_adjoint_map_matches_oracle(torch, solver):
    from gpu_util import to_dev, to_host
    wl = _case()
    disc = _set(solver, wl)
    M = dense.operator_matrix(disc)
    nu = W.random_density(disc.N, 3)
    y = to_host(solver.matvec_adjoint(to_dev(torch, nu)))
    ref = M.conj().T @ nu
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    mu = W.random_density(disc.N, 4)
    Amu = to_host(solver.matvec(to_dev(torch, mu)))
    dual = abs(np.vdot(nu, Amu) - np.vdot(y, mu)) / abs(np.vdot(nu, Amu))
    print("adjoint map vs oracle M^H: %.2e; <nu, A mu> - <A^H nu, mu>: %.2e" % (err, dual))
    assert err <= 1e-12 and dual <= 1e-12


def test_adjoint_solve(torch, solver):
    """GMRES on the conjugate-transpose system: the returned nu satisfies it
    (residual formed independently with the adjoint map) and equals the oracle's
    solve of M^H nu = r."""
    from gpu_util import to_dev, to_host
    wl = _case()
    disc = _set(solver, wl)
    r = W.random_density(disc.N, 5)
    nu, info = solver.solve(b=to_dev(torch, r), tol=1e-12, max_iter=1000, adjoint=True)
    res = np.linalg.norm(to_host(solver.matvec_adjoint(nu)) - r) / np.linalg.norm(r)
    M = dense.operator_matrix(disc)
    ref = np.linalg.solve(M.conj().T, r)
    err = np.linalg.norm(to_host(nu) - ref) / np.linalg.norm(ref)
    print("adjoint solve: %d iterations, residual %.2e (reported %.2e), vs oracle %.2e" %
          (info["iters"], res, info["rel_residual"], err))
    assert info["converged"] and res <= 1e-12 and err <= 1e-10


def _weights(n):
    return np.linspace(1.0, 2.0, n)


def test_objective_and_adjoint_rhs_match_oracle(torch, solver):
    """J = sum_n w_n e_n equals the oracle's; the right-hand side is
    conj(sum_n w_n (beta_n / beta) conj(B_n) c_n), with c_n the oracle's
    coefficient vectors (B_n of unit densities)."""
    from gpu_util import to_dev, to_host
    wl = _case()
    disc = _set(solver, wl)
    mu = W.random_density(disc.N, 6)
    orders = rayleigh.propagating_orders(disc.k, disc.alpha, disc.d)
    w = _weights(len(orders))
    J, rhs = solver.objective_adjoint_rhs(to_dev(torch, mu), w)
    B = rayleigh.rayleigh_coefficients(disc, mu, orders)
    bn = np.real(rayleigh.beta_of(disc.k, rayleigh.alpha_n(disc.alpha, disc.d, orders)))
    s = w * bn / disc.beta
    J_o = float(np.sum(s * np.abs(B) ** 2))
    C = np.stack([rayleigh.rayleigh_coefficients(disc, np.eye(disc.N)[l], orders) for l in range(disc.N)], 1)
    g = (s * np.conj(B)) @ C
    err = np.linalg.norm(to_host(rhs) - np.conj(g)) / np.linalg.norm(g)
    print("J %.12f (oracle %.12f); adjoint rhs vs oracle %.2e" % (J, J_o, err))
    assert abs(J - J_o) <= 1e-12 * abs(J_o) and err <= 1e-12


def _oracle_J(wl, a, b, w):
    disc = dense.Discretization(wl.with_(a_coef=tuple(a), b_coef=tuple(b)))
    M = dense.operator_matrix(disc)
    n, e, _ = rayleigh.efficiencies(disc, np.linalg.solve(M, dense.rhs(disc)))
    return float(np.sum(w * e))


def _gpu_J(solver, wl, a, b, w):
    _set(solver, wl, a, b)
    mu, _ = solver.solve(tol=1e-13, max_iter=1000, allow_noconv=True)
    return solver.objective_adjoint_rhs(mu, w)[0]


def _fd(Jfun, a0, b0, kind, m, h):
    ap, bp, am, bm = a0.copy(), b0.copy(), a0.copy(), b0.copy()
    (ap if kind == "a" else bp)[m] += h
    (am if kind == "a" else bm)[m] -= h
    return (Jfun(ap, bp) - Jfun(am, bm)) / (2 * h)


def _richardson(Jfun, a0, b0, kind, m):
    """central differences at steps 2e-3 and 1e-3, extrapolated (error O(h^4))"""
    return (4 * _fd(Jfun, a0, b0, kind, m, 1e-3) - _fd(Jfun, a0, b0, kind, m, 2e-3)) / 3


def test_shape_gradient_vs_finite_differences(torch, solver):
    """dJ/da_m and dJ/db_m (m = 0..2) by the adjoint against finite
    differences of the objective: central differences with step 1e-6 (noise-
    limited at ~1e-7 by the solves' rounding) and Richardson-extrapolated
    central differences (steps 2e-3, 1e-3) of the library's own solves for
    every coefficient, and Richardson-extrapolated differences of the oracle's
    objective (dense LU + efficiencies) for a_1 and b_2."""
    wl = _case()
    disc = _set(solver, wl)
    orders = rayleigh.propagating_orders(disc.k, disc.alpha, disc.d)
    w = _weights(len(orders))
    mu, _ = solver.solve(tol=1e-13, max_iter=1000, allow_noconv=True)
    J, rhs = solver.objective_adjoint_rhs(mu, w)
    nu, info = solver.solve(b=rhs, tol=1e-13, max_iter=1000, adjoint=True, allow_noconv=True)
    ga, gb = solver.shape_gradient(mu, nu, w, 2)
    a0, b0 = np.array(wl.a_coef, dtype=float), np.array(wl.b_coef, dtype=float)
    Jg = lambda a, b: _gpu_J(solver, wl, a, b, w)  # noqa: E731
    scale = max(np.max(np.abs(ga)), np.max(np.abs(gb)))
    e6, er = 0.0, 0.0
    for m in range(3):
        for kind, g in (("a", ga[m]), ("b", gb[m])):
            if kind == "b" and m == 0:
                continue
            e6 = max(e6, abs(_fd(Jg, a0, b0, kind, m, 1e-6) - g) / scale)
            er = max(er, abs(_richardson(Jg, a0, b0, kind, m) - g) / scale)
    print("J %.10f; adjoint grad a %s b %s" % (J, np.array2string(ga, precision=10), np.array2string(gb, precision=10)))
    print("vs GPU finite differences: step 1e-6 %.2e, Richardson %.2e (relative to max|grad|)" % (e6, er))
    assert e6 <= 1e-6 and er <= 1e-8
    # the oracle's objective (dense LU), two coefficients
    Jo = lambda a, b: _oracle_J(wl, a, b, w)  # noqa: E731
    for kind, m, g in (("a", 1, ga[1]), ("b", 2, gb[2])):
        fo = _richardson(Jo, a0, b0, kind, m)
        print("oracle finite differences d J / d %s_%d = %.12f, adjoint %.12f" % (kind, m, fo, g))
        assert abs(fo - g) <= 1e-8 * scale


def test_deep_corrugation_gradient(torch, solver):
    """The deep-corrugation workload (256 Fourier coefficients, 10 lambda peak
    to peak, period 10 lambda) at N = 2048: the gradient of the specular
    efficiency with respect to all 256 cosine coefficients by one adjoint
    solve, against Richardson-extrapolated finite differences of the library's
    own solves for the three largest entries and one of the smallest; energy
    balance holds.  (The set-up keeps the derivative matrices: the one-pass
    assembly on this geometry; the finite differences use plain set-ups.)"""
    wl = W.config_c5(2048)
    disc = _set(solver, wl, adjoint=1)
    mu, info = solver.solve(tol=1e-11, max_iter=3000, allow_noconv=True)
    n, e, eps = solver.efficiencies(mu)
    w = np.zeros(len(n))
    w[list(n).index(0)] = 1.0
    J, rhs = solver.objective_adjoint_rhs(mu, w)
    nu, _ = solver.solve(b=rhs, tol=1e-12, max_iter=3000, adjoint=True, allow_noconv=True)
    ga, gb = solver.shape_gradient(mu, nu, w, 256)
    a0, b0 = np.array(wl.a_coef, dtype=float), np.array(wl.b_coef, dtype=float)

    def Jg(a, b):
        _set(solver, wl, a, b)
        m_, _ = solver.solve(tol=1e-11, max_iter=3000, allow_noconv=True)
        return solver.objective_adjoint_rhs(m_, w)[0]

    scale = np.max(np.abs(ga))
    idx = list(np.argsort(-np.abs(ga[1:]))[:3] + 1) + [200]
    errs = [abs(_richardson(Jg, a0, b0, "a", m) - ga[m]) / scale for m in idx]
    print("deep profile N = 2048: %d iterations, eps %.1e, e_0 %.6f; d e_0 / d a_m for m = %s: %s; "
          "vs finite differences %s" % (info["iters"], eps, J, idx, np.array2string(ga[idx], precision=6),
                                        ["%.1e" % v for v in errs]))
    assert abs(eps) <= 1e-4 and max(errs) <= 1e-6


def test_autograd_function(torch, solver):
    """The torch.autograd.Function: J.backward() fills the coefficient
    gradients with the adjoint shape gradient."""
    import paper_1707_04950_amd as lib
    wl = _case()
    disc = dense.Discretization(wl)
    orders = rayleigh.propagating_orders(disc.k, disc.alpha, disc.d)
    w = _weights(len(orders))
    a = torch.tensor(wl.a_coef, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(wl.b_coef, dtype=torch.float64, requires_grad=True)
    J = lib.efficiency_objective(solver, a, b, w, _surface_kw(wl, disc), tol=1e-12)
    J.backward()
    _set(solver, wl)
    mu, _ = solver.solve(tol=1e-13, max_iter=1000, allow_noconv=True)
    J2, rhs = solver.objective_adjoint_rhs(mu, w)
    nu, _ = solver.solve(b=rhs, tol=1e-13, max_iter=1000, adjoint=True, allow_noconv=True)
    ga, gb = solver.shape_gradient(mu, nu, w, 2)
    print("autograd J %.12f grad a %s b %s" % (float(J.detach()), a.grad.numpy(), b.grad.numpy()))
    assert abs(float(J.detach()) - J2) <= 1e-11 * abs(J2)
    # (the function's solves stop at 1e-12, the reference ones at 1e-13)
    assert np.allclose(a.grad.numpy(), ga, rtol=0, atol=1e-8 * np.max(np.abs(ga)))
    assert np.allclose(b.grad.numpy(), gb, rtol=0, atol=1e-8 * np.max(np.abs(ga)))


def test_kept_derivative_matrices(torch, solver):
    """sesm_params.adjoint = 1: the operator assembled together with its
    derivative matrices equals the plain assembly (forward maps to rounding),
    and the shape gradient from the kept matrices equals the one that forms
    them on the call; the accelerated mode rejects the flag."""
    import paper_1707_04950_amd as lib
    from gpu_util import set_surface, to_dev, to_host
    wl = _case()
    disc = dense.Discretization(wl)
    orders = rayleigh.propagating_orders(disc.k, disc.alpha, disc.d)
    w = _weights(len(orders))
    m = to_dev(torch, W.random_density(disc.N, 4))
    out = {}
    for flag in (0, 1):
        _set(solver, wl, adjoint=flag)
        y = to_host(solver.matvec(m))
        mu, _ = solver.solve(tol=1e-13, max_iter=1000, allow_noconv=True)
        J, rhs = solver.objective_adjoint_rhs(mu, w)
        nu, _ = solver.solve(b=rhs, tol=1e-13, max_iter=1000, adjoint=True, allow_noconv=True)
        ga, gb = solver.shape_gradient(mu, nu, w, 2)
        out[flag] = (y, np.concatenate([ga, gb]))
    dy = np.max(np.abs(out[1][0] - out[0][0])) / np.max(np.abs(out[0][0]))
    dg = np.max(np.abs(out[1][1] - out[0][1])) / np.max(np.abs(out[0][1]))
    print("kept derivatives: forward map %.2e (bitwise %s), gradient %.2e" %
          (dy, np.array_equal(out[1][0], out[0][0]), dg))
    assert dy <= 1e-14 and dg <= 1e-10
    with pytest.raises(lib.SesmError):
        set_surface(solver, wl, disc, mode=lib.MODE_ACCEL, adjoint=1)


def test_adjoint_arguments(torch, solver):
    import paper_1707_04950_amd as lib
    from gpu_util import set_surface, to_dev
    wl = _case()
    disc = dense.Discretization(wl)
    set_surface(solver, wl, disc, mode=lib.MODE_ACCEL)
    mu = to_dev(torch, W.random_density(disc.N, 1))
    with pytest.raises(lib.SesmError):
        solver.matvec_adjoint(mu)
    with pytest.raises(lib.SesmError):
        solver.solve(b=mu, adjoint=True)
    _set(solver, wl)
    with pytest.raises(lib.SesmError):
        solver.solve(adjoint=True)  # no right-hand side
    with pytest.raises(lib.SesmError):
        solver.objective_adjoint_rhs(mu, [1.0])  # one weight per propagating order
