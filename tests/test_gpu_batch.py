"""GPU tests of the batched forward map (sesm_matvec_batch, Algorithm 3 for
several densities with one operator).

* A batch reproduces single forward maps bit for bit (accelerated and dense
  modes, batch sizes that leave every remainder of the four-density groups,
  padded leading dimensions whose padding stays untouched).
* The batched map agrees with the oracle's accelerated map and with its
  dense direct operator, also at N = 32768 on the sampled rows stored by
  tests/golden/gen_rows_grazing32768.py.
* Densities whose Bloch wavenumbers differ by 2 pi / d share the operator
  (eq. shifted_periodic_green_function depends on alpha only through
  e^{i alpha d}; the completion set of eq. M_eta only through {alpha_n}).
* Degenerate calls: nrhs = 0, negative nrhs, a leading dimension below N,
  overlapping spans, no surface.
"""
import ctypes
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import accel, dense

pytestmark = pytest.mark.gpu

ACC_KW = dict(L=0.5, n_s=10, n_e=1, n_coll=60, n_plw=32)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _gauss30(theta_deg=30.0):
    a, b = W.gaussian_surface(5.0, 0.5, 1.0, W.SEED_BASE + 5)
    return W.Workload(name="gauss30", d=5.0, k=2 * math.pi, theta_deg=theta_deg, N=400, j=8, h=0.85, A=40.0,
                      a_coef=a, b_coef=b, L=0.5)


def _configure(solver, wl, disc, accelerated, **kw):
    from gpu_util import set_surface
    import paper_1707_04950_amd as lib
    if accelerated:
        set_surface(solver, wl, disc, mode=lib.MODE_ACCEL, n_side=ACC_KW["n_s"], n_ext=ACC_KW["n_e"],
                    n_coll=ACC_KW["n_coll"], n_plw=ACC_KW["n_plw"], **kw)
    else:
        set_surface(solver, wl, disc, mode=lib.MODE_DENSE)


def _densities(torch, N, seeds, pad=0):
    """(len(seeds), N + pad) device tensor whose first N columns hold the
    seeded densities and whose padding holds a sentinel."""
    host = np.full((len(seeds), N + pad), 7.0 - 3.0j)
    for r, s in enumerate(seeds):
        host[r, :N] = W.random_density(N, s)
    return torch.from_numpy(host).cuda()


@pytest.mark.parametrize("accelerated", [True, False])
@pytest.mark.parametrize("nrhs,pad", [(1, 0), (3, 5), (4, 0), (7, 3), (9, 0)])
def test_batch_equals_single_bitwise(torch, solver, accelerated, nrhs, pad):
    wl = _gauss30()
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, accelerated)
    N = disc.N
    mu = _densities(torch, N, list(range(11, 11 + nrhs)), pad)
    out = torch.full((nrhs, N + pad), complex(-5.0, 2.0), dtype=torch.complex128, device="cuda")
    solver.matvec_batch(mu[:, :N], out[:, :N])
    torch.cuda.synchronize()
    for r in range(nrhs):
        y1 = solver.matvec(mu[r, :N].contiguous())
        assert torch.equal(out[r, :N], y1), "density %d of %d differs from the single forward map" % (r, nrhs)
    if pad:
        assert bool((out[:, N:] == complex(-5.0, 2.0)).all()), "padding of the outputs was written"
        assert bool((mu[:, N:] == complex(7.0, -3.0)).all())


def test_batch_vs_oracle(torch, solver):
    """Rows of a batch against the oracle's accelerated map (same algorithm
    and parameters) and its dense direct operator (method error)."""
    from gpu_util import to_host
    wl = _gauss30()
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    seeds = [1, 2, 3, 4, 5]
    mu = _densities(torch, disc.N, seeds)
    Y = to_host(solver.matvec_batch(mu))
    op = accel.AccelOperator(disc, **ACC_KW)
    M = dense.operator_matrix(disc)
    for r, s in enumerate(seeds):
        m = W.random_density(disc.N, s)
        y_acc, y_den = op.matvec(m), M @ m
        e_acc = np.linalg.norm(Y[r] - y_acc) / np.linalg.norm(y_acc)
        e_den = np.linalg.norm(Y[r] - y_den) / np.linalg.norm(y_den)
        print("density %d: rel err vs oracle accel %.2e, vs oracle dense %.2e" % (r, e_acc, e_den))
        assert e_acc <= 1e-9
        assert e_den <= 1e-8


def test_batch_full_size_grazing_wood(torch, solver):
    """N = 32768 near-grazing Wood workload, in the launch configuration the
    benchmark times (groups of four densities): a batch of six equals single
    forward maps bit for bit, and its third row (seed 5) matches the oracle's
    64 stored rows to the accelerator's tolerance."""
    import paper_1707_04950_amd as lib
    wl = W.config_grazing_wood(32768)
    disc = dense.Discretization(wl)
    with open(os.path.join(GOLDEN, "rows_grazing32768.json")) as fh:
        G = json.load(fh)
    assert G["N"] == disc.N and G["n_a"] == disc.n_a and G["workload"] == wl.name
    solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, wl.j, wl.A, disc.N,
                       h=wl.h, c=wl.c, n_a=disc.n_a, gamma_frac=wl.gamma_frac, eta=wl.eta, mode=lib.MODE_ACCEL,
                       L=wl.L)
    seeds = [21, 22, 5, 23, 24, 25]
    mu = _densities(torch, disc.N, seeds)
    Y = solver.matvec_batch(mu)
    torch.cuda.synchronize()
    for r in range(len(seeds)):
        assert torch.equal(Y[r], solver.matvec(mu[r].contiguous())), "density %d differs" % r
    rows = np.asarray(G["rows"])
    ref = np.asarray(G["y_re"]) + 1j * np.asarray(G["y_im"])
    y = Y[2].cpu().numpy()
    rel = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
    print("batched row 2, 64 sampled rows: max rel err vs oracle %.2e" % rel)
    assert rel <= 1e-8


@pytest.mark.parametrize("accelerated", [True, False])
def test_bloch_class_shares_operator(torch, solver, accelerated):
    """Incidences with alpha' = alpha - 2 pi / d: the surface set up for
    either gives the same forward map (up to rounding of the tables).  At 37
    degrees the completion set is {-8, 2}, and {-7, 3} for alpha'."""
    wl = _gauss30(37.0)
    s1 = math.sin(math.radians(37.0)) - 2 * math.pi / (wl.k * wl.d)
    wl2 = _gauss30(math.degrees(math.asin(s1)))
    assert abs(wl2.alpha - (wl.alpha - 2 * math.pi / wl.d)) < 1e-12
    mu = _densities(torch, wl.N, [31, 32, 33])
    Y, U = [], []
    for w in (wl, wl2):
        disc = dense.Discretization(w)
        _configure(solver, w, disc, accelerated)
        U.append(solver.info()["U_eta"])
        Y.append(solver.matvec_batch(mu).cpu().numpy())
    assert len(U[0]) > 0 and list(U[1]) == [n + 1 for n in U[0]], U
    rel = np.max(np.abs(Y[0] - Y[1])) / np.max(np.abs(Y[0]))
    print("accelerated" if accelerated else "dense", "alpha vs alpha - 2 pi/d: max rel diff %.2e" % rel)
    assert rel <= 1e-10


def test_batch_timing_counts(torch, solver):
    """Kernel timing of a batch of six densities (groups of four and two): each
    later stage is one launch per group carrying the bytes of all its
    densities; the shared first launch is not timed.  (The single forward
    map keeps every near-field item in its first launch here, as the batch
    does, so that the later stages carry the same bytes.)"""
    import paper_1707_04950_amd as lib
    wl = _gauss30()
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True, near_split=-1)
    mu = _densities(torch, disc.N, [51])
    solver.timing_enable((1 << lib.KT_COUNT) - 1)
    solver.matvec(mu[0])
    one = solver.timing_read()
    solver.timing_enable((1 << lib.KT_COUNT) - 1)
    solver.matvec_batch(_densities(torch, disc.N, list(range(52, 58))))
    st = solver.timing_read()
    solver.timing_enable(0)
    assert st["k_local_apply"]["launches"] == 0
    for k in ("k_merge_fft", "k_fft_rows", "k_yconv", "k_cells_far"):
        assert st[k]["launches"] == 2, k
        assert st[k]["bytes"] == pytest.approx(6 * one[k]["bytes"], rel=1e-12), k


def test_batch_degenerate_calls(torch, solver):
    import paper_1707_04950_amd as lib
    wl = _gauss30()
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    N = disc.N
    f = solver.lib.sesm_matvec_batch
    mu = _densities(torch, N, [1, 2])
    out = torch.zeros((2, N), dtype=torch.complex128, device="cuda")
    pm, po = ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert f(solver.h, 0, None, 0, None, 0) == 0                     # nothing to do
    assert f(solver.h, -1, pm, N, po, N) == lib.SESM_EINVAL           # negative count
    assert f(solver.h, 2, pm, N - 1, po, N) == lib.SESM_EINVAL        # leading dimension below N
    assert f(solver.h, 2, pm, N, po, N - 1) == lib.SESM_EINVAL
    assert f(solver.h, 2, None, N, po, N) == lib.SESM_EINVAL          # null pointer
    assert f(solver.h, 2, pm, N, pm, N) == lib.SESM_EINVAL            # same span
    half = ctypes.c_void_p(mu.data_ptr() + 16 * N)                    # outputs start inside the densities
    assert f(solver.h, 1, pm, N, half, N) == 0                        # density 0 and row 1: disjoint
    assert f(solver.h, 2, pm, N, half, N) == lib.SESM_EINVAL          # overlapping spans
    torch.cuda.synchronize()
    assert bool((out == 0).all())
    with pytest.raises(ValueError):
        solver.matvec_batch(mu[:, : N - 1])
    fresh = lib.Solver(0)
    try:
        assert fresh.lib.sesm_matvec_batch(fresh.h, 1, pm, N, po, N) == lib.SESM_ENOSURF
    finally:
        fresh.close()


# ---- batched solve (sesm_solve_batch) and Bloch-class right-hand sides

def _bloch_member(wl, p):
    """The workload of the incidence alpha + 2 pi p / d (same surface)."""
    s1 = math.sin(math.radians(wl.theta_deg)) + 2 * math.pi * p / (wl.k * wl.d)
    return wl.with_(theta_deg=math.degrees(math.asin(s1)))


@pytest.mark.parametrize("accelerated", [True, False])
def test_solve_batch_equals_single_solves(torch, solver, accelerated):
    """Four Bloch-class incidences, a zero and a random right-hand side
    (groups of four and two): every solution and iteration count equals
    the single unrestarted solve's bit for bit."""
    wl = _gauss30(37.0)
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, accelerated)
    N = disc.N
    rows = [solver.rhs_bloch(p) for p in (0, -1, -3, 1)]
    rows.append(torch.zeros(N, dtype=torch.complex128, device="cuda"))
    rows.append(_densities(torch, N, [61])[0])
    B = torch.stack(rows)
    assert torch.equal(B[0], solver.rhs())
    tol = 1e-9 if accelerated else 1e-12  # (accelerated: above its rounding floor)
    mu, infos = solver.solve_batch(B, tol=tol, max_iter=400)
    for r in range(B.shape[0]):
        m1, i1 = solver.solve(B[r].contiguous(), tol=tol, max_iter=400)
        print("member %d: iters %d (single %d), residual %.2e" % (r, infos[r]["iters"], i1["iters"],
                                                                  infos[r]["rel_residual"]))
        assert infos[r]["converged"] and infos[r]["column_mismatches"] == 0
        assert infos[r]["iters"] == i1["iters"] and infos[r]["rel_residual"] == i1["rel_residual"]
        assert torch.equal(mu[r], m1), "solution %d differs from the single solve" % r
    assert infos[4]["iters"] == 0 and bool((mu[4] == 0).all())


def test_solve_batch_single_member(torch, solver):
    """A batch of one (one-member launches throughout) equals the single solve."""
    wl = _gauss30(37.0)
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    B = solver.rhs_bloch(-1)[None, :]
    mu, infos = solver.solve_batch(B, tol=1e-9, max_iter=400)
    m1, i1 = solver.solve(B[0].contiguous(), tol=1e-9, max_iter=400)
    assert infos[0]["converged"] and infos[0]["iters"] == i1["iters"] and torch.equal(mu[0], m1)


def test_solve_batch_bloch_efficiencies_vs_oracle(torch, solver):
    """Members p = 0, -1, 1 of the Bloch class of the 37 degree incidence,
    solved in one accelerated batch: the right-hand sides equal the oracle's
    for each incidence, and the efficiencies (taken on a surface set up for
    that incidence) and their energy balance match the dense oracle solved
    for it to 1e-6."""
    from gpu_util import to_host
    from oracle import rayleigh
    wl = _gauss30(37.0)
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    ps = (0, -1, 1)
    B = torch.stack([solver.rhs_bloch(p) for p in ps])
    mu, infos = solver.solve_batch(B, tol=1e-9, max_iter=400)
    M = dense.operator_matrix(disc)
    for r, p in enumerate(ps):
        wp = _bloch_member(wl, p)
        dp = dense.Discretization(wp)
        b_o = dense.rhs(dp)
        assert np.max(np.abs(to_host(B[r]) - b_o)) < 1e-12
        n_o, e_o, eps_o = rayleigh.efficiencies(dp, np.linalg.solve(M, b_o))
        _configure(solver, wp, dp, True)
        n, e, eps = solver.efficiencies(mu[r])
        err = float(np.max(np.abs(e - e_o)))
        print("p = %d: %d orders, max|e - e_oracle| %.2e, energy balance %.2e (oracle %.2e)"
              % (p, len(n), err, eps, eps_o))
        # the energy balance at N = 400 is the discretisation's (oracle alike)
        assert list(n) == list(n_o) and err <= 1e-6 and abs(eps - eps_o) <= 1e-6


def test_solve_batch_arguments(torch, solver):
    import paper_1707_04950_amd as lib
    wl = _gauss30(37.0)
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    N = disc.N
    f = solver.lib.sesm_solve_batch
    b = _densities(torch, N, [1, 2])
    x = torch.zeros((2, N), dtype=torch.complex128, device="cuda")
    pb, px = ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr())
    assert f(solver.h, 0, None, 0, None, 0, 1e-10, 10, 0, None) == 0
    assert f(solver.h, lib.SESM_MAX_BATCH + 1, pb, N, px, N, 1e-10, 10, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, -1, pb, N, px, N, 1e-10, 10, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, pb, N, px, N, 1e-10, 0, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, pb, N, px, N, 1e-10, 4001, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, pb, N, px, N, 0.0, 10, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, pb, N - 1, px, N, 1e-10, 10, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, None, N, px, N, 1e-10, 10, 0, None) == lib.SESM_EINVAL
    assert f(solver.h, 2, pb, N, pb, N, 1e-10, 10, 0, None) == lib.SESM_EINVAL
    torch.cuda.synchronize()
    assert bool((x == 0).all())
    # a cap too small to converge: soft failure, outputs and records written
    xs, infos = solver.solve_batch(b, tol=1e-14, max_iter=3, allow_noconv=True)
    assert all(i["iters"] == 3 and not i["converged"] for i in infos) and bool(torch.isfinite(xs).all())
    with pytest.raises(lib.SesmError):
        solver.rhs_bloch(2)  # alpha + 4 pi / d > k at 37 degrees and d = 5
    fresh = lib.Solver(0)
    try:
        assert fresh.lib.sesm_solve_batch(fresh.h, 1, pb, N, px, N, 1e-10, 10, 0, None) == lib.SESM_ENOSURF
        assert fresh.lib.sesm_rhs_bloch(fresh.h, 0, px) == lib.SESM_ENOSURF
    finally:
        fresh.close()


def test_solve_batch_full_size_grazing_wood(torch, solver):
    """N = 32768 near-grazing Wood workload, members p = 0, -1, -2 in one
    batch: member 0 equals the single solve bit for bit; every member's
    efficiencies (surface set up for its incidence) balance energy to 1e-6."""
    import paper_1707_04950_amd as lib
    wl = W.config_grazing_wood(32768)
    disc = dense.Discretization(wl)

    def setup(w):
        solver.set_surface(np.asarray(w.a_coef), np.asarray(w.b_coef), w.d, w.k, w.alpha, w.j, w.A, disc.N,
                           h=w.h, c=w.c, n_a=disc.n_a, gamma_frac=w.gamma_frac, eta=w.eta, mode=lib.MODE_ACCEL,
                           L=w.L)
    setup(wl)
    ps = (0, -1, -2)
    B = torch.stack([solver.rhs_bloch(p) for p in ps])
    # members p != 0 have |mu| / |b| ~ 600, which puts their true-residual
    # floor near 2e-8
    mu, infos = solver.solve_batch(B, tol=5e-8, max_iter=3000)
    m0, i0 = solver.solve(tol=5e-8, max_iter=3000)
    assert torch.equal(mu[0], m0) and infos[0]["iters"] == i0["iters"]
    for r, p in enumerate(ps):
        setup(_bloch_member(wl, p))
        n, e, eps = solver.efficiencies(mu[r])
        print("p = %d: %d iterations, %d orders, energy balance %.2e" % (p, infos[r]["iters"], len(n), eps))
        assert infos[r]["converged"] and infos[r]["column_mismatches"] == 0 and abs(eps) <= 1e-6


@pytest.mark.parametrize("nrhs,pad", [(1, 0), (5, 3), (8, 0), (9, 2), (17, 0)])
def test_batch_matrix_cores_match_single(torch, solver, nrhs, pad):
    """batch_mfma = 1: the near field of up to eight densities per pass on the
    FP64 matrix cores.  Every row equals its single forward map to rounding
    (the sums run in another order: not bit for bit), the padding stays
    untouched."""
    wl = _gauss30()
    disc = dense.Discretization(wl)
    _configure(solver, wl, disc, True)
    N = disc.N
    mu = _densities(torch, N, list(range(31, 31 + nrhs)), pad)
    ys = torch.stack([solver.matvec(mu[r, :N].contiguous()) for r in range(nrhs)])
    _configure(solver, wl, disc, True, batch_mfma=1)
    out = torch.full((nrhs, N + pad), complex(-5.0, 2.0), dtype=torch.complex128, device="cuda")
    solver.matvec_batch(mu[:, :N], out[:, :N])
    torch.cuda.synchronize()
    err = float((out[:, :N] - ys).abs().max() / ys.abs().max())
    print("nrhs %d: matrix-core batch vs single maps %.2e" % (nrhs, err))
    assert err <= 1e-14
    if pad:
        assert bool((out[:, N:] == complex(-5.0, 2.0)).all())


def test_incidence_set_matrix_cores(torch, solver):
    """Incidence sets (different alpha per member) with batch_mfma = 1: each
    member's forward map equals the vector-unit one to rounding."""
    wl = _gauss30()
    disc = dense.Discretization(wl)
    alphas = [wl.k * math.sin(math.radians(t)) for t in (5.0, 17.0, 30.0, 44.0, 61.0)]
    mu = _densities(torch, disc.N, list(range(51, 56)))
    _configure(solver, wl, disc, True)
    solver.set_incidences(alphas)
    yv = solver.matvec_incidences(mu)
    _configure(solver, wl, disc, True, batch_mfma=1)
    solver.set_incidences(alphas)
    ym = solver.matvec_incidences(mu)
    err = float((ym - yv).abs().max() / yv.abs().max())
    print("incidence set, matrix cores vs vector units: %.2e" % err)
    assert err <= 1e-14
