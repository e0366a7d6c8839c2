"""Pins of the oracle's off-surface field (oracle/field.py) against facts
outside it: the exact reflected wave of a flat surface, the field of a
quasi-periodic point source below the surface whose Dirichlet data are
imposed (the exterior solution is that field itself), the Rayleigh expansion
built from the separately pinned coefficients, and quasi-periodicity.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, field, greens


def _solve(wl, rhs=None):
    disc = dense.Discretization(wl)
    M = dense.operator_matrix(disc)
    b = dense.rhs(disc) if rhs is None else rhs(disc)
    return disc, np.linalg.solve(M, b)


@pytest.mark.parametrize("offset", [0.0, 0.3])
def test_flat_surface_reflected_wave(offset):
    """f = const: the scattered field above the plane is the reflected wave
    -e^{-2 i beta f} e^{i (alpha x + beta y)} (Dirichlet condition)."""
    wl = W.config_dense_sinusoid(64).with_(a_coef=(offset,), b_coef=(0.0,), A=40.0)
    disc, mu = _solve(wl)
    X = np.array([0.1, 0.9, 1.7, 2.4, -3.1])
    Y = offset + np.array([0.3, 0.5, 0.8, 1.2, 2.0])
    u = field.scattered_field(disc, mu, X, Y)
    ex = -np.exp(-2j * disc.beta * offset) * np.exp(1j * (disc.alpha * X + disc.beta * Y))
    err = np.max(np.abs(u - ex))
    print("flat offset %.1f: max |u - u_exact| %.2e" % (offset, err))
    assert err < 1e-8


def _ptsrc(k, alpha, d, X, Y, nmax=300):
    out = 0
    for n in range(-nmax, nmax + 1):
        an = alpha + 2 * np.pi * n / d
        bn = greens.beta_of(k, np.array([an]))[0]
        out = out + 1j / (2 * d * bn) * np.exp(1j * an * X + 1j * bn * np.abs(Y))
    return out


def test_point_source_field_is_reproduced():
    """Dirichlet data of a quasi-periodic point source below the surface: the
    scattered field above the surface is the source's own field, at points
    between the crests (inside the surface's height range) and above it."""
    wl = W.config_dense_sinusoid(128).with_(A=40.0)
    x0, y0 = 0.7, -0.8
    disc, mu = _solve(wl, rhs=lambda D: _ptsrc(D.k, D.alpha, D.d, D.x - x0, D.f - y0))
    X = np.array([0.0, 0.6, 1.25, 1.9, 2.2])
    fX = 0.125 * disc.d * np.cos(2 * np.pi * X / disc.d)
    Y = fX + np.array([0.25, 0.4, 0.3, 0.6, 1.0])  # 6 to 25 node spacings above the curve
    u = field.scattered_field(disc, mu, X, Y)
    ex = _ptsrc(disc.k, disc.alpha, disc.d, X - x0, Y - y0)
    err = np.max(np.abs(u - ex)) / np.max(np.abs(ex))
    print("point source: max rel err %.2e" % err)
    assert err < 1e-5


def test_rayleigh_expansion_equals_direct_field():
    """Above max f the Rayleigh expansion (exact lattice sums, all orders up
    to a decay cut) and the direct rule (windowed lattice sums) agree up to the
    window's truncation error, which falls with the window half-width A:
    6.8e-7 at A = 40 periods, 1.5e-11 at A = 160 (same density)."""
    wl = W.config_dense_sinusoid(128).with_(A=40.0)
    disc, mu = _solve(wl)
    fmax = float(np.max(disc.f))
    X = np.array([0.2, 1.1, 2.3])
    Y = fmax + np.array([0.15, 0.4, 1.0])
    nmax = int(math.ceil((40.0 / 0.15) * disc.d / (2 * math.pi))) + 5
    r = field.rayleigh_field(disc, mu, X, Y, nmax)
    errs = []
    for A in (40.0, 160.0):
        u = field.scattered_field(dense.Discretization(wl.with_(A=A)), mu, X, Y)
        errs.append(np.max(np.abs(u - r)) / np.max(np.abs(u)))
    print("direct (A = 40, 160) vs Rayleigh: %.2e %.2e" % tuple(errs))
    assert errs[0] < 2e-6 and errs[1] < 1e-9


def test_field_is_quasi_periodic():
    wl = W.config_dense_sinusoid(64).with_(A=40.0)
    disc, mu = _solve(wl)
    X = np.array([0.3, 1.4])
    Y = np.array([0.9, 0.6])
    u0 = field.scattered_field(disc, mu, X, Y)
    u1 = field.scattered_field(disc, mu, X + disc.d, Y)
    assert np.max(np.abs(u1 - np.exp(1j * disc.alpha * disc.d) * u0)) < 1e-9 * np.max(np.abs(u0))
