"""Off-surface field (sesm_field) through the C ABI against the oracle's
direct rule and Rayleigh expansion (oracle/field.py, pinned on a flat
surface, a manufactured point source and the Rayleigh coefficients), in both
modes and on every route of the accelerated mode (cell grid, Rayleigh
expansion, direct rule), plus the flat-surface closed form and
quasi-periodicity on the GPU itself.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, field

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


def _prof(wl, x):
    a, b = np.asarray(wl.a_coef), np.asarray(wl.b_coef)
    m = np.arange(len(a))
    out = a[0] + np.sum(a[None, 1:] * np.cos(2 * np.pi * m[None, 1:] * x[:, None] / wl.d), 1)
    if len(b) > 1:
        out += np.sum(b[None, 1:len(a)] * np.sin(2 * np.pi * m[None, 1:len(b)] * x[:, None] / wl.d), 1)
    return out


def _solve(solver, wl, mode, tol):
    from gpu_util import set_surface, to_host
    disc = dense.Discretization(wl)
    set_surface(solver, wl, disc, mode=mode)
    mu, info = solver.solve(tol=tol, max_iter=1000, allow_noconv=True)
    print("  solve: %d iterations, true residual %.2e" % (info["iters"], info["rel_residual"]))
    assert info["rel_residual"] <= 5 * tol  # (the accelerated map's rounding floor; any density serves the field)
    return disc, mu, to_host(mu)


def test_dense_field_matches_oracle(torch, solver):
    """Dense mode (direct rule at every point) on the sinusoid: points between
    the crests, far above, and outside the first period."""
    import paper_1707_04950_amd as lib
    from gpu_util import to_host
    wl = W.config_dense_sinusoid(256)
    disc, mu, mu_h = _solve(solver, wl, lib.MODE_DENSE, 1e-11)
    X = np.array([0.05, 0.7, 1.3, 2.0, 2.45, -1.1, 4.2, 0.9])
    Y = _prof(wl, X) + np.array([0.06, 0.1, 0.25, 0.5, 1.0, 0.3, 0.2, 3.0])
    u = to_host(solver.field(mu, X, Y))
    ref = field.scattered_field(disc, mu_h, X, Y)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print("dense field vs oracle: max rel err %.2e" % err)
    assert err <= 1e-11


def _accel_case():
    a, b = W.gaussian_surface(5.0, 0.5, 1.0, W.SEED_BASE + 5)
    return W.Workload(name="gauss-d5", d=5.0, k=2 * math.pi, theta_deg=30.0, N=400, j=8, h=0.5, A=40.0, a_coef=a,
                      b_coef=b, L=0.5)


def test_accel_field_routes_match_oracle(torch, solver):
    """Accelerated mode on a random surface: points inside the cell grid
    (above the curve by at least 5 dx), points above the grid (Rayleigh
    expansion) and points between the grid top and max f + L/4 (direct rule),
    each against the oracle's counterpart for the same density."""
    import paper_1707_04950_amd as lib
    from gpu_util import to_host
    wl = _accel_case()
    disc, mu, mu_h = _solve(solver, wl, lib.MODE_ACCEL, 1e-8)
    inf = solver.info()
    y0, L, ny = inf["y0"], inf["L"], inf["n_y"]
    ytop, fmax = y0 + ny * L, float(np.max(disc.f))
    rng = np.random.default_rng(7)
    # inside the grid, above the curve
    Xg = rng.uniform(-wl.d, 2 * wl.d, 40)
    fg = _prof(wl, Xg)
    lo = fg + 5 * disc.dx
    ok = lo < ytop - 1e-3
    Xg, lo = Xg[ok], lo[ok]
    Yg = lo + rng.uniform(0, 1, len(Xg)) * (ytop - 1e-3 - lo)
    # above the grid: Rayleigh route, and the band between the grid top and max f + L/4 when there is one
    Xr = rng.uniform(0, wl.d, 6)
    Yr = max(ytop, fmax + 0.25 * L) + np.array([0.0, 0.05, 0.2, 0.5, 1.0, 2.0])
    u_g = to_host(solver.field(mu, Xg, Yg))
    u_r = to_host(solver.field(mu, Xr, Yr))
    ref_g = field.scattered_field(disc, mu_h, Xg, Yg)
    nR = int(math.ceil((math.sqrt((40 / (Yr.min() - fmax)) ** 2 + wl.k ** 2) + wl.k) * wl.d / (2 * math.pi))) + 2
    ref_r = field.rayleigh_field(disc, mu_h, Xr, Yr, nR)
    eg = np.max(np.abs(u_g - ref_g)) / np.max(np.abs(ref_g))
    er = np.max(np.abs(u_r - ref_r)) / np.max(np.abs(ref_r))
    print("grid route: %d points, max rel err %.2e; Rayleigh route: max rel err %.2e" % (len(Xg), eg, er))
    # grid route: the accelerator's interpolation error (the plane-wave fit of
    # the cells' far fields; 3.7e-8 measured), Rayleigh route: rounding
    assert len(Xg) >= 10 and eg <= 1e-7 and er <= 1e-10
    if fmax + 0.25 * L > ytop + 1e-3:  # the direct route
        Xd = rng.uniform(0, wl.d, 4)
        Yd = ytop + (fmax + 0.25 * L - ytop) * np.array([0.1, 0.4, 0.7, 0.95])
        u_d = to_host(solver.field(mu, Xd, Yd))
        ref_d = field.scattered_field(disc, mu_h, Xd, Yd)
        ed = np.max(np.abs(u_d - ref_d)) / np.max(np.abs(ref_d))
        print("direct route: max rel err %.2e" % ed)
        assert ed <= 1e-11


def test_accel_field_flat_surface_closed_form(torch, solver):
    """f = 0.2 (flat): above the plane the scattered field is the reflected
    wave -e^{-2 i beta f} e^{i (alpha x + beta y)}, on the grid and Rayleigh
    routes of the accelerated mode."""
    import paper_1707_04950_amd as lib
    from gpu_util import to_host
    wl = _accel_case().with_(a_coef=(0.2,), b_coef=(0.0,))
    disc, mu, _ = _solve(solver, wl, lib.MODE_ACCEL, 1e-10)
    inf = solver.info()
    ytop = inf["y0"] + inf["n_y"] * inf["L"]
    X = np.array([0.3, 1.7, 3.9, -2.2, 7.4, 0.8])
    Y = np.array([0.2 + 6 * disc.dx, 0.2 + 0.5 * (ytop - 0.2), ytop - 1e-3, ytop + 0.3, 1.5, 3.0])
    u = to_host(solver.field(mu, X, Y))
    ex = -np.exp(-2j * disc.beta * 0.2) * np.exp(1j * (disc.alpha * X + disc.beta * Y))
    err = np.max(np.abs(u - ex))
    print("flat surface: max |u - exact| %.2e" % err)
    assert err <= 1e-8


def test_field_quasi_periodic_and_routes_continuous(torch, solver):
    """u(x + p d, y) = e^{i alpha p d} u(x, y) on the grid route, to the
    rounding of the wrapped abscissa (x + p d - p d differs from x in the last
    bits, and the cells' plane-wave weights, large and cancelling, carry that
    difference up to ~1e-9); at the grid top the grid route and the route above
    it agree."""
    import paper_1707_04950_amd as lib
    from gpu_util import to_host
    wl = _accel_case()
    disc, mu, _ = _solve(solver, wl, lib.MODE_ACCEL, 1e-8)
    inf = solver.info()
    ytop = inf["y0"] + inf["n_y"] * inf["L"]
    X = np.array([0.4, 2.1, 4.6])
    Y = np.full(3, ytop - 0.05)
    u0 = to_host(solver.field(mu, X, Y))
    for p in (-2, 1, 3):
        up = to_host(solver.field(mu, X + p * wl.d, Y))
        assert np.max(np.abs(up - np.exp(1j * wl.alpha * wl.d * p) * u0)) <= 1e-8 * np.max(np.abs(u0))
    ua = to_host(solver.field(mu, X, np.full(3, ytop - 1e-9)))
    ub = to_host(solver.field(mu, X, np.full(3, ytop + 1e-9)))
    gap = np.max(np.abs(ua - ub)) / np.max(np.abs(ua))
    print("grid top: inside vs above %.2e" % gap)
    assert gap <= 1e-7  # accelerator error, plus the window error when the route above is the Rayleigh one


def test_field_arguments(torch, solver):
    import paper_1707_04950_amd as lib
    wl = _accel_case()
    disc, mu, _ = _solve(solver, wl, lib.MODE_ACCEL, 1e-8)
    with pytest.raises(lib.SesmError):
        solver.field(mu, [0.1, float("nan")], [1.0, 1.0])
    assert solver.field(mu, [], []).numel() == 0
