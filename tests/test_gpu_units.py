"""GPU unit tests of building blocks and method-parameter invariance.

* The library's own mixed-radix FFT (Sec. 5.5.1, periodic grid direction)
  against NumPy's FFT, for lengths exercising every radix and row batching.
* The library's own phase factor e^{it} (plane-wave exponentials) against
  NumPy's, to a few units in the last place.
* Efficiencies are physical quantities: the accelerated solution must give the
  oracle's efficiencies whatever the method's free parameters (shift h, cell
  side L, equivalent-source density n_s), within the accelerator tolerance.
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def solver(torch):
    import paper_1707_04950_amd as lib
    s = lib.Solver(0)
    yield s
    s.close()


@pytest.mark.parametrize("n,rows", [(2000, 26), (200, 246), (360, 7), (150, 1), (6, 333), (1, 5), (1024, 3)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_own_fft_matches_numpy(torch, solver, n, rows, sign):
    rng = np.random.default_rng(n * 7 + rows)
    x = rng.standard_normal((rows, n)) + 1j * rng.standard_normal((rows, n))
    y = solver.diag_fft(torch.from_numpy(x), sign).cpu().numpy()
    ref = np.fft.fft(x, axis=1) if sign < 0 else np.fft.ifft(x, axis=1) * n
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    assert err < 1e-14 * max(1.0, math.log2(n)) * 4, err


def test_fft_rejects_bad_lengths(torch, solver):
    import paper_1707_04950_amd as lib
    x = torch.zeros((2, 7), dtype=torch.complex128)
    with pytest.raises(lib.SesmError):
        solver.diag_fft(x)  # 7 is not 5-smooth


def test_own_phase_factor_matches_numpy(torch, solver):
    """The library's e^{it} (reduction modulo pi/2, Taylor polynomials) against
    numpy at dense small arguments, near multiples of pi/4, and large ones."""
    rng = np.random.default_rng(17)
    k = np.arange(-400, 401)
    t = np.concatenate([np.linspace(-8.0, 8.0, 20001), k * (np.pi / 4), k * (np.pi / 4) + 1e-9,
                        rng.uniform(-1e4, 1e4, 20000), [0.0, -0.0, 1e-300, 5e-324, 1e-8, -1e-8]])
    got = solver.diag_cexp(torch.from_numpy(t)).cpu().numpy()
    ref = np.exp(1j * t)
    err = np.max(np.abs(got - ref))
    print("max |e^{it} - numpy| %.2e" % err)
    assert err <= 6e-16
    assert np.all(np.abs(np.abs(got) - 1.0) <= 4e-16)


@pytest.mark.parametrize("kw", [dict(h=0.85), dict(h=0.6), dict(L=0.4), dict(n_side=12), dict(j=6), dict(j=10),
                                dict(A=30.0)])
def test_efficiencies_invariant_under_method_parameters(torch, solver, kw):
    """30 degree double-Wood workload (N = 4096): accelerated efficiencies
    against the oracle's (tests/golden/wood30_4096.json, dense LU at h = 0.85,
    j = 8, A = 20 periods), also with another shift order j and window A."""
    import json
    import paper_1707_04950_amd as lib
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "wood30_4096.json")))
    wl = W.config_random_double_wood(4096)
    L = kw.get("L", wl.L)
    n_a = max(8, int(math.floor(0.8 * min(L, wl.d) / wl.dx)))
    solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, kw.get("j", wl.j),
                       kw.get("A", wl.A), wl.N,
                       h=kw.get("h", wl.h), c=wl.c, n_a=n_a, gamma_frac=wl.gamma_frac, eta=wl.eta,
                       mode=lib.MODE_ACCEL, L=L, n_side=kw.get("n_side", 0))
    # above the accelerated map's rounding floor, which rises with the number
    # of equivalent sources per side (a worse-conditioned fit)
    mu, info = solver.solve(tol=2e-7 if kw.get("n_side", 10) > 10 else 1e-8, max_iter=2000)
    n, e, eps = solver.efficiencies(mu)
    assert list(n) == G["orders"]
    err = float(np.max(np.abs(e - np.asarray(G["efficiencies"]))))
    print(kw, "iters", info["iters"], "max|e - e_oracle| %.2e" % err, "eps %.2e" % eps)
    assert err <= 1e-6
