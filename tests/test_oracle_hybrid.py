"""Pins of the oracle's spectral route to G~_j (Sec. 3.2): the series of eq.
(shifted_quasi_per_rayleigh) written in the form of eq. (betan_taylor)
(greens.qper_spectral), its row rule for the hybrid kernel tables
(greens.hybrid_row_order) and the hybrid tables of oracle/accel.py.

Independent routes: the plain spectral series (away from Wood anomalies), the
closed forms of the beta-quotients (against their Taylor sums), the windowed
spatial lattice sums (which converge to the exact G~_j as the window grows, at
the algebraic rate the paper states at Wood anomalies), and continuity in the
incidence across a Wood anomaly.
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads as W  # noqa: E402
from oracle import accel, dense, greens  # noqa: E402

K0 = 2 * math.pi


def _plain(kind, k, alpha, d, j, h, X, Y, nmax):
    if kind == "mono":
        return greens.lattice_sum_spectral(k, alpha, d, j, h, X, Y, nmax)
    dH = greens.lattice_sum_spectral(k, alpha, d, j, h, X, Y, nmax, kernel="dl", fps=0.0)  # -dG/dY
    if kind == "dipH":
        return dH
    return dH - greens.lattice_sum_spectral(k, alpha, d, j, h, X, Y, nmax, kernel="dl", fps=1.0)  # -dG/dX


@pytest.mark.parametrize("kind", ["mono", "dipH", "dipV"])
def test_wood_safe_series_equals_plain_series(kind):
    """Away from Wood anomalies the rewritten series is the printed one, at
    heights above, between and below the shifted pole rows."""
    k, d, j, h = K0, 5.0, 8, 0.85
    alpha = k * math.sin(math.radians(30.0))
    X = np.linspace(0.0, d, 7, endpoint=False) + 0.01
    for Y in (0.3, -0.4, -1.3, 2.0, -5.5):
        a = greens.qper_spectral(k, alpha, d, j, h, X, Y, 200, kind)
        b = _plain(kind, k, alpha, d, j, h, X, Y, 200)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), (kind, Y)


@pytest.mark.parametrize("beta", [0.1, 0.3, 0.49, 0.2j, 0.45j, 0.3 + 0.1j, 1e-7j, 1e-9])
def test_beta_quotients_match_closed_forms(beta):
    """The Taylor sums used for small |beta| equal the closed forms
    (1 - e^{i beta h})^j / beta and (e^{i beta t} - e^{-i beta t}) / beta."""
    h, j, t = 0.85, 8, -1.7
    closed_pow = (-np.expm1(1j * beta * h)) ** j / beta  # (expm1 keeps the digits of a tiny beta)
    closed_odd = 2j * np.sin(beta * t) / beta
    assert abs(greens._q_pow(beta, h, j) - closed_pow) <= 1e-14 * max(abs(closed_pow), 1e-300)
    assert abs(greens._q_odd(beta, t) - closed_odd) <= 1e-14 * abs(closed_odd)


def test_series_equals_windowed_sums_off_wood():
    """Eq. (Gq_limit) with a long window equals the spectral series at
    points off the pole rows (an independent route through Hankel functions)."""
    k, d, j, h = K0, 1.3, 3, 0.4
    alpha = k * math.sin(math.radians(20.0))
    X = np.array([0.1, 0.45, 0.9, 1.2])
    for kind, kern in (("mono", "G"), ("dipH", "dl")):
        sp = np.concatenate([greens.qper_spectral(k, alpha, d, j, h, X, Y, 80, kind)
                             for Y in (0.25, -0.3, -0.7, -1.05)])
        ss = np.concatenate([greens.lattice_sum_windowed(k, alpha, d, j, h, 400 * d, 0.5, X, np.full_like(X, Y),
                                                         kernel=kern, fps=0.0) for Y in (0.25, -0.3, -0.7, -1.05)])
        assert np.max(np.abs(sp - ss)) < 1e-7 * np.max(np.abs(sp)), kind


def _wood_case():
    d, j, h, theta, n0 = 5.0, 8, 0.85, 30.0, 8
    k = 2 * math.pi * n0 / (d * (1 + math.sin(math.radians(theta))))  # alpha_{-n0} = -k: beta_{-n0} = 0
    return k, k * math.sin(math.radians(theta)), d, j, h, n0


def test_windowed_sums_converge_to_series_at_wood():
    """At a Wood anomaly the series stays finite and the windowed sums reach
    it algebraically in the window half-width A (the appendix's A^{-3.5} rate
    for j = 8): each doubling of A from 25 to 200 periods brings them more than
    8x closer, and at A = 200 periods they agree to ~1e-8."""
    k, alpha, d, j, h, n0 = _wood_case()
    assert abs(greens.beta_of(k, alpha - 2 * math.pi * n0 / d)) < 1e-6
    X = np.linspace(0.0, d, 9, endpoint=False) + 0.013
    for Y in (0.37, -0.61):
        for kind, kern in (("mono", "G"), ("dipH", "dl")):
            ref = greens.qper_spectral(k, alpha, d, j, h, X, Y, 400, kind)
            assert np.all(np.isfinite(ref))
            errs = []
            for A in (25, 50, 100, 200):
                w = greens.lattice_sum_windowed(k, alpha, d, j, h, A * d, 0.5, X, np.full_like(X, Y), kernel=kern,
                                                fps=0.0)
                errs.append(np.max(np.abs(w - ref)))
            print(Y, kind, ["%.2e" % e for e in errs])
            assert all(errs[i] > 8 * errs[i + 1] for i in range(3))
            assert errs[-1] < 5e-8 * np.max(np.abs(ref))


def test_series_is_continuous_across_wood():
    """The series at incidences a hair off the Wood anomaly (beta_{-n0} of
    order 1e-4, real or imaginary) differs from the value at the anomaly by
    O(|alpha - alpha_W|)."""
    k, alpha, d, j, h, n0 = _wood_case()
    X = np.array([0.2, 1.7, 3.3])
    for kind in ("mono", "dipH", "dipV"):
        g0 = greens.qper_spectral(k, alpha, d, j, h, X, -0.61, 300, kind)
        for da in (1e-9, -1e-9):
            g1 = greens.qper_spectral(k, alpha + da, d, j, h, X, -0.61, 300, kind)
            assert np.max(np.abs(g1 - g0)) < 1e-6 * np.max(np.abs(g0)), (kind, da)


def test_row_rule_truncation_and_pole_rows():
    """Pole rows (Y = -m h) keep the windowed sums; elsewhere the order the rule
    picks leaves a tail below 1e-15 of the row (the series at twice the order
    agrees)."""
    k, d, j, h = K0, 5.0, 8, 0.85
    alpha = k * math.sin(math.radians(47.0))
    assert greens.hybrid_row_order(k, d, j, h, -3 * h) is None
    assert greens.hybrid_row_order(k, d, j, h, 0.0) is None
    X = np.linspace(0.0, d, 11, endpoint=False)
    for Y in (0.05, -0.4, -2.5):
        nm = greens.hybrid_row_order(k, d, j, h, Y)
        assert nm is not None
        for kind in ("mono", "dipH"):
            a = greens.qper_spectral(k, alpha, d, j, h, X, Y, nm, kind)
            b = greens.qper_spectral(k, alpha, d, j, h, X, Y, 2 * nm, kind)
            assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b)), (Y, kind, nm)


def test_hybrid_tables_equal_long_window_tables():
    """The hybrid kernel tables of the accelerated oracle: spectral rows equal
    the windowed tables of a 400-period window (off Wood), spatial rows are the
    windowed sums of a window 8 times as wide as the table's (here 8 x 50 = 400
    periods); both grids and both kernels (H: monopole and d/dy2 dipole; V:
    d/dx2 dipole), on the small pin geometry."""
    a, b = W.gaussian_surface(3.0, 0.4, 1.0, W.SEED_BASE + 11)
    wl = W.Workload(name="hyb-pin", d=3.0, k=K0, theta_deg=20.0, N=240, j=8, h=0.5, A=50.0,
                    a_coef=a, b_coef=b, L=0.5)
    assert accel.HYBRID_WINDOW == 8.0
    g = accel.Geometry(dense.Discretization(wl))
    g400 = accel.Geometry(dense.Discretization(wl.with_(A=400.0)))
    for lam in ("H", "V"):
        for kind in ("mono", "dip" + lam):
            Tw = accel.lattice_table(g400, lam, kind, "windowed")
            Th = accel.lattice_table(g, lam, kind, "hybrid")
            hy = g.L if lam == "H" else g.delta
            nY = (Tw.shape[0] + 1) // 2
            rows = [r for r in range(Tw.shape[0])
                    if greens.hybrid_row_order(wl.k, wl.d, wl.j, wl.h, (r - nY + 1) * hy) is not None]
            assert 0 < len(rows) < Tw.shape[0]
            other = [r for r in range(Tw.shape[0]) if r not in rows]
            assert np.array_equal(Th[other], Tw[other])
            err = np.max(np.abs(Th[rows] - Tw[rows])) / np.max(np.abs(Tw[rows]))
            print(lam, kind, "spectral rows", len(rows), "of", Tw.shape[0], "max rel diff %.2e" % err)
            assert err < 1e-8
