"""Independent NumPy brute force of the one-dimensional SPFM (TI + h3) step.

TEST INFRASTRUCTURE ONLY.  Written separately from ``spfm_oracle.c``: it uses
the 1D form of the discrete energy (Eq. 1 with a single direction, |r| = dx,
gamma_1 nu_1 = 1) and obtains g'(phi) by complex-step differentiation of Eq. 6
as printed, not from a closed-form derivative.  With n = [100] the coupling
parameter of Eq. 5 is a = tanh(2 dx / lambda).

Scheme (Eq. 2, forward Euler in time, periodic in x):
    dF_i = Gamma/(C_Gamma lambda) [ g'(phi_i) - lambda^2 (phi_{i+1} - 2 phi_i + phi_{i-1}) / dx^2 ]
           + mu * 6 phi_i (1 - phi_i)
    phi_i <- phi_i - dt * 2 M / (3 lambda Gamma) * dF_i
"""
from __future__ import annotations

import numpy as np


def g_eq6(phi, a: float, rho: float, lam: float):
    """Eq. 6 exactly as printed; works on complex arguments."""
    q = a * a
    u = 1.0 - 2.0 * phi
    return lam * lam / (rho * rho) * (phi * (1.0 - phi)
                                      + (1.0 - q) / (4.0 * q) * np.log((1.0 - q) / (1.0 - q * u * u)))


def g_prime_complex_step(phi, a: float, rho: float, lam: float, h: float = 1e-30):
    """d g / d phi of Eq. 6 by the complex-step method, Im g(phi + i h) / h."""
    return np.imag(g_eq6(np.asarray(phi, dtype=np.complex128) + 1j * h, a, rho, lam)) / h


def rate(phi: np.ndarray, *, dx=1.0, lam=4.0, Gamma=1.0, M=1.0, mu=0.0, C_Gamma=2.0 / 3.0):
    a = np.tanh(2.0 * dx / lam)
    lap = np.roll(phi, -1) - 2.0 * phi + np.roll(phi, 1)
    dF = Gamma / (C_Gamma * lam) * (g_prime_complex_step(phi, a, dx, lam) - lam * lam * lap / (dx * dx)) \
        + mu * 6.0 * phi * (1.0 - phi)
    return -2.0 * M / (3.0 * lam * Gamma) * dF


def run(phi0: np.ndarray, nsteps: int, *, dt=0.1, **kw) -> np.ndarray:
    phi = np.array(phi0, dtype=np.float64, copy=True)
    for _ in range(int(nsteps)):
        phi = phi + dt * rate(phi, **kw)
    return phi


def ideal_profile(x: np.ndarray, c: float, lam: float) -> np.ndarray:
    """Eq. 3 with n = [100]: phi = (1 - tanh(2 (x - c)/lambda)) / 2."""
    return 0.5 * (1.0 - np.tanh(2.0 * (x - c) / lam))
