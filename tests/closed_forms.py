"""Closed forms and independent numerical solutions that pin the oracle.

None of these re-types the Monte Carlo method: each is an analytic result or a
deterministic solution of the corresponding integral / differential equation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

HBAR = 1.054571817e-34
KB = 1.380649e-23


def En(n: int, x):
    return special.expn(n, x)


def gray_slab_integral_equation(tau_L: float, n: int = 2000):
    """Gray slab between black walls (non-dimensional emissive power phi, flux Psi).

    phi(tau) = 1/2 [E2(tau) + int_0^tau_L phi(t) E1(|tau - t|) dt],
    Psi = 1 - 2 int_0^tau_L phi(t) E2(t) dt  (Heaslet-Warming form of the gray slab).
    Solved by product integration: phi piecewise constant on n cells, collocation at the
    midpoints, E1 integrated exactly through E2 (E2' = -E1), and E2 through E3.
    Returns (cell edges in optical depth, phi per cell, Psi).
    """
    t = np.linspace(0.0, tau_L, n + 1)
    mid = 0.5 * (t[:-1] + t[1:])
    a = mid[:, None]
    lo = t[None, :-1]
    hi = t[None, 1:]
    K = np.where(a >= hi, En(2, np.maximum(a - hi, 0)) - En(2, np.maximum(a - lo, 0)),
                 np.where(a <= lo, En(2, np.maximum(lo - a, 0)) - En(2, np.maximum(hi - a, 0)), 0.0))
    idx = np.arange(n)
    h = t[1] - t[0]
    K[idx, idx] = 2.0 * (1.0 - En(2, 0.5 * h))
    A = np.eye(n) - 0.5 * K
    phi = np.linalg.solve(A, 0.5 * En(2, mid))
    Psi = 1.0 - 2.0 * np.sum(phi * (En(3, t[:-1]) - En(3, t[1:])))
    return t, phi, Psi


def fs_suppression(delta: float, p: float = 0.0) -> float:
    """Fuchs-Sondheimer in-plane suppression, delta = d / Lambda, wall specularity p:
    S = 1 - 3 (1 - p)/(2 delta) int_1^inf (t^-3 - t^-5)(1 - e^{-delta t})/(1 - p e^{-delta t}) dt."""
    f = lambda t: (t ** -3 - t ** -5) * (-math.expm1(-delta * t)) / (1.0 - p * math.exp(-delta * t))
    val, _ = integrate.quad(f, 1.0, np.inf, limit=400, epsabs=1e-14, epsrel=1e-12)
    return 1.0 - 1.5 * (1.0 - p) / delta * val


def ballistic_transient_dT(z, t, L, v, dT_l, dT_r):
    """Ballistic temperature between two walls switched on at t = 0 (the paper's ballistic
    benchmark, Eq. Analytical_T)."""
    z = np.asarray(z, dtype=float)
    a = 1.0 - z / (v * t)
    b = 1.0 - (L - z) / (v * t)
    return 0.5 * a * (a > 0) * dT_l + 0.5 * b * (b > 0) * dT_r


def bin_average(f, lo: float, hi: float, nbins: int, per_bin: int = 64):
    """Average of f over each of nbins equal bins of [lo, hi] (Gauss-Legendre per bin)."""
    x, wq = np.polynomial.legendre.leggauss(per_bin)
    edges = np.linspace(lo, hi, nbins + 1)
    out = np.zeros(nbins)
    for i in range(nbins):
        a, b = edges[i], edges[i + 1]
        z = 0.5 * (b - a) * x + 0.5 * (a + b)
        out[i] = 0.5 * np.sum(wq * f(z))
    return out


def fourier_neumann_piecewise(z, t, D, L, edges, dT, n_images: int = 6):
    """Heat equation on [0, L] with insulated ends, initial condition piecewise constant
    (value dT[c] on [edges[c], edges[c+1])), by the method of images."""
    z = np.asarray(z, dtype=float)
    s = math.sqrt(4.0 * D * t)
    out = np.zeros_like(z)
    a, b = edges[:-1], edges[1:]
    for nimg in range(-n_images, n_images + 1):
        sh = 2.0 * nimg * L
        for lo, hi in ((a + sh, b + sh), (-b + sh, -a + sh)):
            out += np.sum(dT[None, :] * 0.5 * (special.erf((z[:, None] - lo[None, :]) / s)
                                               - special.erf((z[:, None] - hi[None, :]) / s)), axis=1)
    return out


def bose_einstein_energy(omega, T):
    """Equilibrium energy per mode hbar omega / (exp(hbar omega / k_B T) - 1)."""
    x = HBAR * omega / (KB * T)
    return HBAR * omega / math.expm1(x)


def dispersion_integrals(T: float, omega_max=(7.5e13, 3.0e13), g=(1.0, 2.0), a_si=5.431e-10,
                         A=1.3e-45, B=1.7e-19, Cc=137.0):
    """Heat capacity and kinetic kappa of the continuous sine dispersion, integrated in k
    (D d omega = g k^2 / (2 pi^2) dk, so the integrand is smooth up to the zone edge)."""
    k_max = 2.0 * math.pi / a_si
    a_eff = math.pi / k_max
    Ctot = 0.0
    kap = 0.0
    for wm, gg in zip(omega_max, g):
        def cw(k):
            w = wm * math.sin(0.5 * a_eff * k)
            x = HBAR * w / (KB * T)
            h = 0.5 * x
            return gg * k * k / (2 * math.pi ** 2) * KB * h * h / math.sinh(h) ** 2

        def kw(k):
            w = wm * math.sin(0.5 * a_eff * k)
            v = 0.5 * a_eff * wm * math.cos(0.5 * a_eff * k)
            tau = 1.0 / (A * w ** 4 + B * w * w * T * math.exp(-Cc / T))
            return cw(k) * v * v * tau / 3.0

        Ctot += integrate.quad(cw, 0.0, k_max, limit=200, epsrel=1e-12)[0]
        kap += integrate.quad(kw, 0.0, k_max, limit=400, epsrel=1e-10)[0]
    return Ctot, kap
