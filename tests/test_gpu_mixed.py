"""Mixed precision (FP32 EqSources operators and FP32 Krylov bases under FP64
iterative refinement; near field, quadratures, lattice sums and every sum in
FP64): the FP64 true residual reaches the tolerance and the efficiencies
match the oracle's and the plain FP64 solve's."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import dense, rayleigh

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def _set(solver, wl, N=None, mixed=1):
    import paper_1707_04950_amd as lib
    disc = dense.Discretization(wl, N=N)
    solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, wl.j, wl.A, disc.N,
                       h=wl.h, c=wl.c, n_a=disc.n_a, gamma_frac=wl.gamma_frac, eta=wl.eta, mode=lib.MODE_ACCEL,
                       L=wl.L, mixed=mixed)
    return disc


@pytest.mark.parametrize("name,factory,tol", [("wood30_4096", W.config_random_double_wood, 1e-9)])
def test_mixed_solve_matches_fp64_and_oracle(torch, solver, name, factory, tol):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        G = json.load(fh)
    wl = factory(G["N"])
    _set(solver, wl)
    mu64, i64 = solver.solve(tol=tol, max_iter=3000)
    mu32, i32 = solver.solve(tol=tol, max_iter=3000, mixed=True)
    b = solver.rhs()
    r = float(torch.linalg.vector_norm(b - solver.matvec(mu32)) / torch.linalg.vector_norm(b))
    _, e64, _ = solver.efficiencies(mu64)
    n, e32, eps = solver.efficiencies(mu32)
    d64 = float(np.max(np.abs(e32 - e64)))
    dor = float(np.max(np.abs(e32 - np.asarray(G["efficiencies"]))))
    print("%s: FP64 %d iterations; mixed %d iterations in %d refinement steps, FP64 true residual %.2e "
          "(independent %.2e); max|e_mixed - e_fp64| %.2e, vs oracle %.2e" %
          (name, i64["iters"], i32["iters"], i32["residual_restarts"], i32["rel_residual"], r, d64, dor))
    assert i32["converged"] and i32["rel_residual"] <= tol and abs(i32["rel_residual"] - r) <= 1e-3 * r
    assert d64 <= 1e-7 and dor <= 1e-6




def test_mixed_incidence_batch(torch, solver):
    """Mixed precision for a batch of incidences (three Bloch classes) in
    lockstep: each member's FP64 residual reaches tol and its efficiencies
    match the dense oracle's."""
    thetas = (20.0, 30.0, 47.0)
    a, b = W.gaussian_surface(5.0, 0.5, 1.0, W.SEED_BASE + 5)
    mk = lambda t: W.Workload(name="g5", d=5.0, k=2 * math.pi, theta_deg=t, N=400, j=8, h=0.85, A=40.0,  # noqa: E731
                              a_coef=a, b_coef=b, L=0.5)
    _set(solver, mk(30.0))
    solver.set_incidences([mk(t).alpha for t in thetas])
    X64, i64 = solver.solve_incidences(tol=1e-8, max_iter=600)
    X32, i32 = solver.solve_incidences(tol=1e-8, max_iter=600, mixed=True)
    for r, t in enumerate(thetas):
        disc = dense.Discretization(mk(t))
        M = dense.operator_matrix(disc)
        n_o, e_o, _ = rayleigh.efficiencies(disc, np.linalg.solve(M, dense.rhs(disc)))
        n, e, eps = solver.efficiencies_incidence(r, X32[r].contiguous())
        _, e6, _ = solver.efficiencies_incidence(r, X64[r].contiguous())
        print("theta %4.1f: FP64 %d it; mixed %d it, %d steps, residual %.2e; vs FP64 %.2e, vs oracle %.2e" %
              (t, i64[r]["iters"], i32[r]["iters"], i32[r]["residual_restarts"], i32[r]["rel_residual"],
               np.max(np.abs(e - e6)), np.max(np.abs(e - e_o))))
        assert i32[r]["converged"] and np.max(np.abs(e - e6)) <= 1e-7 and np.max(np.abs(e - e_o)) <= 1e-6


def test_mixed_needs_fp32_operators(torch, solver):
    import paper_1707_04950_amd as lib
    wl = W.config_random_double_wood(4096)
    _set(solver, wl, mixed=0)
    with pytest.raises(lib.SesmError):
        solver.solve(tol=1e-8, max_iter=100, mixed=True)


def test_mixed_grazing_stagnation_is_reported(torch, solver):
    """On the near-grazing Wood workload (N = 4096, |mu| / |b| ~ 120) the FP32
    bases cannot carry the inner solves: the refinement stops when the FP64
    residual no longer halves and the solve reports non-convergence with its
    true FP64 residual (soft error; mu and the record are written)."""
    wl = W.config_grazing_wood(4096)
    _set(solver, wl)
    mu, info = solver.solve(tol=1e-8, max_iter=1500, allow_noconv=True, mixed=True)
    b = solver.rhs()
    r = float(torch.linalg.vector_norm(b - solver.matvec(mu)) / torch.linalg.vector_norm(b))
    print("grazing, mixed: %d iterations, %d refinement steps, residual %.2e (independent %.2e), converged %s" %
          (info["iters"], info["residual_restarts"], info["rel_residual"], r, info["converged"]))
    assert abs(info["rel_residual"] - r) <= 1e-3 * r and bool(torch.isfinite(mu).all())
    assert info["converged"] == (r <= 1e-8)
