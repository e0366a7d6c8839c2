"""GPU parity of the dense direct path against the oracle (through the C ABI)."""
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


@pytest.fixture(scope="module")
def c1():
    wl = W.config_dense_sinusoid(256)
    disc = dense.Discretization(wl)
    M = dense.operator_matrix(disc)
    return wl, disc, M


def test_hankel_functions_vs_mpmath(torch, solver):
    import mpmath
    mpmath.mp.dps = 30
    x = np.concatenate([np.geomspace(1e-3, 4.99, 120), [5.0, 5.0 + 1e-12], np.geomspace(5.01, 40, 120),
                        np.geomspace(40, 3e4, 80)])
    h0, h1 = solver.diag_hankel(torch.from_numpy(x))
    h0, h1 = h0.cpu().numpy(), h1.cpu().numpy()
    for t, xv in enumerate(x):
        r0 = complex(mpmath.hankel1(0, xv))
        r1 = complex(mpmath.hankel1(1, xv))
        # rounding of x itself perturbs the phase by ~ x * 2^-53
        tol = 2e-14 + 4e-16 * xv
        assert abs(h0[t] - r0) <= tol * abs(r0), (xv, h0[t], r0)
        assert abs(h1[t] - r1) <= tol * abs(r1), (xv, h1[t], r1)


def test_info_matches_oracle(solver, c1):
    from gpu_util import set_surface
    wl, disc, M = c1
    set_surface(solver, wl, disc)
    inf = solver.info()
    assert inf["N"] == disc.N and inf["n_a"] == disc.n_a
    assert sorted(inf["U_eta"]) == sorted(disc.U_eta.tolist())
    U = rayleigh.propagating_orders(disc.k, disc.alpha, disc.d)
    assert inf["n_first"] == U[0] and inf["n_count"] == len(U)


def test_rhs_parity(torch, solver, c1):
    from gpu_util import set_surface, to_host
    wl, disc, M = c1
    set_surface(solver, wl, disc)
    b = to_host(solver.rhs())
    assert np.max(np.abs(b - dense.rhs(disc))) < 1e-13


def test_dense_matvec_parity_sinusoid(torch, solver, c1):
    """Full N = 256 operator, seeded complex density: element-wise parity."""
    from gpu_util import set_surface, to_dev, to_host
    wl, disc, M = c1
    set_surface(solver, wl, disc)
    for seed in (1, 2):
        mu = W.random_density(disc.N, seed)
        y = to_host(solver.matvec(to_dev(torch, mu)))
        ref = M @ mu
        assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))
    # a plane wave exp(i alpha_n x), the structure the operator diagonalises on flat surfaces
    mu = np.exp(1j * (disc.alpha - 2 * np.pi / disc.d) * disc.x)
    y = to_host(solver.matvec(to_dev(torch, mu)))
    assert np.max(np.abs(y - M @ mu)) <= 1e-11 * np.max(np.abs(M @ mu))


def test_dense_solve_and_efficiencies_sinusoid(torch, solver, c1):
    from gpu_util import set_surface, to_host
    wl, disc, M = c1
    set_surface(solver, wl, disc)
    mu, info = solver.solve(tol=1e-12, max_iter=200)
    assert info["converged"]
    mu_ref = np.linalg.solve(M, dense.rhs(disc))
    mu = to_host(mu)
    assert np.max(np.abs(mu - mu_ref)) < 1e-9 * np.max(np.abs(mu_ref))
    n, e, eps = solver.efficiencies(solver.solve(tol=1e-12, max_iter=200)[0])
    n_o, e_o, eps_o = rayleigh.efficiencies(disc, mu_ref)
    assert np.array_equal(n, n_o)
    assert np.max(np.abs(e - e_o)) < 1e-10
    assert abs(eps - eps_o) < 1e-10


@pytest.mark.parametrize("N,kw", [(100, dict(theta_deg=20.0, n_a=16)),         # ragged N, other angle
                                  (72, dict(j=0, A=30.0, n_a=12)),              # unshifted kernel
                                  (96, dict(j=3, h=0.41, n_a=15))])             # odd j, other h
def test_dense_matvec_parity_ragged(torch, solver, N, kw):
    from gpu_util import set_surface, to_dev, to_host
    wl = W.config_dense_sinusoid(N).with_(**kw)
    disc = dense.Discretization(wl)
    set_surface(solver, wl, disc)
    mu = W.random_density(N, 7)
    rows = np.array([0, 1, N // 3, N // 2, N - 2, N - 1])
    ref = dense.operator_rows(disc, rows) @ mu
    y = to_host(solver.matvec(to_dev(torch, mu)))
    assert np.max(np.abs(y[rows] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_flat_surface_at_wood_closed_form(torch, solver):
    """Flat surface exactly at a Wood anomaly: B_0 = -1 (closed form)."""
    from gpu_util import set_surface
    d, th = 2.5, 30.0
    wl = W.config_dense_sinusoid(64).with_(a_coef=(0.0,), b_coef=(0.0,), A=40.0, theta_deg=th,
                                           k=W.wood_grazing_k(d, th, 1))
    disc = dense.Discretization(wl)
    set_surface(solver, wl, disc)
    assert -1 in solver.info()["U_eta"]
    mu, info = solver.solve(tol=1e-12, max_iter=100)
    B = solver.rayleigh(mu, [0, -1])
    assert abs(B[0] + 1) < 1e-6


def test_errors_are_reported(torch, solver):
    import paper_1707_04950_amd as lib
    wl = W.config_dense_sinusoid(64)
    with pytest.raises(lib.SesmError) as ei:
        solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, 1.2 * wl.k, 8, 20.0, 64)
    assert ei.value.code == lib.SESM_EINVAL
    with pytest.raises(lib.SesmError) as ei:   # a >= d
        solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, 8, 20.0, 64, n_a=64)
    assert ei.value.code == lib.SESM_EINVAL
    s2 = lib.Solver(0)
    with pytest.raises(lib.SesmError) as ei:
        s2.N = 16
        s2.matvec(s2.empty(), s2.empty())
    assert ei.value.code == lib.SESM_ENOSURF
    s2.close()


@pytest.mark.parametrize("kw,why", [(dict(N=0), "empty discretisation"), (dict(N=4), "fewer than 8 nodes"),
                                    (dict(j=17), "shift order beyond 16"), (dict(A=0.0), "no window"),
                                    (dict(d=-1.0), "negative period"), (dict(mode=7), "unknown mode")])
def test_degenerate_inputs_are_rejected(torch, solver, kw, why):
    """Empty, too small or meaningless inputs are rejected by the host checks
    (no kernel runs), with SESM_EINVAL and a message."""
    import paper_1707_04950_amd as lib
    wl = W.config_dense_sinusoid(64)
    args = dict(d=wl.d, j=wl.j, A=wl.A, N=64)
    extra = {}
    for key, v in kw.items():
        (args if key in args else extra)[key] = v
    with pytest.raises(lib.SesmError) as ei:
        solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), args["d"], wl.k, wl.alpha, args["j"],
                           args["A"], args["N"], **extra)
    assert ei.value.code == lib.SESM_EINVAL, why


def test_solve_arguments_are_validated(torch, solver, c1):
    """A valid surface, then solver arguments outside their ranges: rejected,
    and the context stays usable."""
    import paper_1707_04950_amd as lib
    from gpu_util import set_surface
    wl, disc = c1[0], c1[1]
    set_surface(solver, wl, disc)
    for kw in (dict(tol=0.0), dict(tol=-1.0), dict(max_iter=0), dict(restart=-1)):
        with pytest.raises(lib.SesmError) as ei:
            solver.solve(**{**dict(tol=1e-10, max_iter=50), **kw})
        assert ei.value.code == lib.SESM_EINVAL, kw
    mu, info = solver.solve(tol=1e-10, max_iter=200)
    assert info["converged"]
