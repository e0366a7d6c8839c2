"""Seeded synthetic inputs shared by the CPU oracle and the GPU library tests.

This module holds input recipes only: surface Fourier coefficients, incidence
parameters and seeded density vectors.  It contains none of the scattering
method's arithmetic (no Green functions, quadratures or solvers), so that the
oracle and the HIP path remain independent of each other.

Units: lengths in wavelengths unless stated (lambda = 1, k = 2*pi) except for
the near-grazing workload whose wavenumber is tuned onto a Wood anomaly.

Surface model.  Every profile is a real trigonometric polynomial
    f(x) = a[0] + sum_{m>=1} a[m] cos(2 pi m x / d) + b[m] sin(2 pi m x / d),
the form a periodic surface of period d takes when it is smooth and
band-limited.  Random rough surfaces follow the Gaussian-spectrum model the
paper uses for its randomly rough examples (Sec. 6.4): independent normal
Fourier amplitudes shaped by the Gaussian power spectrum
    W(K) = sigma^2 l_c / (2 sqrt(pi)) * exp(-K^2 l_c^2 / 4),
truncated at K l_c <= 8 and rescaled so the rms height is exactly sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

SEED_BASE = 170704950


@dataclass(frozen=True)
class Workload:
    """One scattering configuration plus discretisation parameters.

    Attributes mirror the symbols of the paper: period ``d``, wavenumber
    ``k``, incidence angle ``theta`` (alpha = k sin theta, beta = k cos
    theta), shift order ``j`` and shift ``h`` of the multipolar Green
    function, window half-width ``A`` in periods with plateau fraction ``c``
    (window S_{cA,A}), singular-window radius ``a = n_a * dx`` with plateau
    ``gamma = gamma_frac * a``, completion threshold ``eta`` and ``N``
    quadrature nodes.  Accelerator parameters: cell side ``L`` and the
    vertical offset of the cell grid.
    """
    name: str
    d: float
    k: float
    theta_deg: float
    N: int
    j: int
    h: float
    A: float
    a_coef: tuple
    b_coef: tuple
    c: float = 0.5
    n_a: int = 0              # 0 -> chosen from L (accelerated) or N (dense)
    gamma_frac: float = 0.5
    eta: float = 1e-3
    L: float = 0.5
    gmres_tol: float = 1e-10

    @property
    def alpha(self) -> float:
        return self.k * math.sin(math.radians(self.theta_deg))

    @property
    def beta(self) -> float:
        return self.k * math.cos(math.radians(self.theta_deg))

    @property
    def dx(self) -> float:
        return self.d / self.N

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def gaussian_surface(d: float, sigma: float, lc: float, seed: int,
                     kmax_lc: float = 8.0):
    """Gaussian-spectrum random periodic surface (cos/sin coefficients).

    Returns (a, b) with a[0] = 0 (zero mean) and rms height exactly sigma.
    """
    rng = np.random.default_rng(seed)
    M = int(math.floor(kmax_lc * d / (2.0 * math.pi * lc)))
    m = np.arange(1, M + 1)
    K = 2.0 * math.pi * m / d
    W = sigma ** 2 * lc / (2.0 * math.sqrt(math.pi)) * np.exp(-(K * lc) ** 2 / 4.0)
    amp = np.sqrt(W * 2.0 * math.pi / d)
    g = rng.standard_normal(M)
    gp = rng.standard_normal(M)
    F = amp * (g + 1j * gp) / math.sqrt(2.0)
    a = np.zeros(M + 1)
    b = np.zeros(M + 1)
    a[1:] = 2.0 * F.real
    b[1:] = -2.0 * F.imag
    rms = math.sqrt(0.5 * float(np.sum(a[1:] ** 2 + b[1:] ** 2)))
    a *= sigma / rms
    b *= sigma / rms
    return tuple(a.tolist()), tuple(b.tolist())


def sinusoid(d: float, amp: float):
    """f(x) = amp * cos(2 pi x / d)."""
    return (0.0, amp), (0.0, 0.0)


def flat(offset: float = 0.0):
    return (offset,), (0.0,)


TWO_PI = 2.0 * math.pi


def config_dense_sinusoid(N: int = 256) -> Workload:
    """Dense direct operator: f = 0.125 d cos(2 pi x/d), d = 2.5 lambda,
    45 degree incidence, j = 8, window of 20 periods."""
    d = 2.5
    a, b = sinusoid(d, 0.125 * d)
    return Workload(name="sinusoid-d2.5-theta45-N%d" % N, d=d, k=TWO_PI,
                    theta_deg=45.0, N=N, j=8, h=0.5, A=20.0,
                    a_coef=a, b_coef=b, n_a=40 * N // 256, L=0.5)


def config_random_double_wood(N: int = 4096) -> Workload:
    """FFT-accelerated FP64 workload: Gaussian random surface, d = 20 lambda,
    rms 0.5 lambda, l_c = 1 lambda, 30 degree incidence (a double Wood
    anomaly: beta_n = 0 for n = 10 and n = -30)."""
    d = 20.0
    a, b = gaussian_surface(d, 0.5, 1.0, SEED_BASE + 2)
    return Workload(name="gauss-d20-rms0.5-theta30-N%d" % N, d=d, k=TWO_PI,
                    theta_deg=30.0, N=N, j=8, h=0.85, A=20.0,
                    a_coef=a, b_coef=b, L=0.5)


def wood_grazing_k(d: float, theta_deg: float, order: int) -> float:
    """Wavenumber with k d (1 + sin theta) / (2 pi) = order (an integer), so
    that alpha_{-order} = -k exactly (Wood anomaly)."""
    return TWO_PI * order / (d * (1.0 + math.sin(math.radians(theta_deg))))


def config_grazing_wood(N: int = 32768) -> Workload:
    """Wood anomaly + near grazing: Gaussian random surface d = 100 lambda,
    rms 1 lambda, l_c = 1 lambda, 89 degree incidence, k tuned so that
    k d (1 + sin theta)/(2 pi) = 200, window of 40 periods."""
    d = 100.0
    a, b = gaussian_surface(d, 1.0, 1.0, SEED_BASE + 3)
    return Workload(name="gauss-d100-rms1-theta89-wood-N%d" % N, d=d,
                    k=wood_grazing_k(d, 89.0, 200), theta_deg=89.0, N=N, j=8,
                    h=0.85, A=40.0, a_coef=a, b_coef=b, L=0.5)


def random_density(N: int, seed: int = 1) -> np.ndarray:
    """Seeded complex normal density vector (complex128)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(N) + 1j * rng.standard_normal(N)) / math.sqrt(2.0)


C4_D_OVER_LAMBDA = (50.0, 50.5, 51.0, 51.5)


def config_c4(i_k: int = 0, N: int = 16384) -> Workload:
    """Many incidences: Gaussian random surface of period d = 50 (units of
    the first wavelength), rms 0.5, l_c = 1, wavenumber k = 2 pi (d/lambda)/d
    for d/lambda in C4_D_OVER_LAMBDA[i_k]; the incidence angle of the returned
    workload is 0 (the set's angles are given by c4_angles)."""
    d = 50.0
    a, b = gaussian_surface(d, 0.5, 1.0, SEED_BASE + 4)
    k = TWO_PI * C4_D_OVER_LAMBDA[i_k] / d
    return Workload(name="gauss-d50-rms0.5-k%d-N%d" % (i_k, N), d=d, k=k, theta_deg=0.0, N=N, j=8, h=0.85,
                    A=40.0, a_coef=a, b_coef=b, L=0.5)


def c4_angles(n: int = 64):
    """n incidence angles uniform in [0, 85] degrees."""
    return [85.0 * i / (n - 1) for i in range(n)]


def deep_profile(d: float, depth: float, n_modes: int, seed: int, m_c: float = 2.0):
    """Deep corrugation: n_modes seeded normal Fourier amplitudes (cos and sin)
    under the envelope exp(-(m / m_c)^2 / 2), scaled so that the profile's
    peak-to-peak depth (on a fine grid) is `depth`; zero mean."""
    rng = np.random.default_rng(seed)
    m = np.arange(1, n_modes + 1)
    env = np.exp(-0.5 * (m / m_c) ** 2)
    a = np.zeros(n_modes + 1)
    b = np.zeros(n_modes + 1)
    a[1:] = env * rng.standard_normal(n_modes)
    b[1:] = env * rng.standard_normal(n_modes)
    x = np.linspace(0.0, d, 8192, endpoint=False)
    f = np.cos(2 * np.pi * np.outer(x, m) / d) @ a[1:] + np.sin(2 * np.pi * np.outer(x, m) / d) @ b[1:]
    scale = depth / (f.max() - f.min())
    return tuple((a * scale).tolist()), tuple((b * scale).tolist())


def config_c5(N: int = 8192, h: float = 0.85, A: float = 80.0) -> Workload:
    """Adjoint-gradient workload: deep corrugation with 256 seeded Fourier
    coefficients (peak-to-peak depth 10 lambda), period 10 lambda, 20 degree
    incidence, j = 8.  The window is 80 periods: at 20 periods the window's
    truncation error leaves an energy-balance error of 2e-2 on this deep
    profile (4e-5 at 40 periods)."""
    d = 10.0
    a, b = deep_profile(d, 10.0, 256, SEED_BASE + 6)
    return Workload(name="deep-d10-pp10-theta20-N%d" % N, d=d, k=TWO_PI, theta_deg=20.0, N=N, j=8, h=h,
                    A=A, a_coef=a, b_coef=b, L=0.5)
