"""Shared helpers of the GPU tests.  Every input field is built by the oracle
(or from the seeded generators), never by the GPU library.

Parity fields.  The TI_n normal n = grad psi / |grad psi| makes the scheme
sensitive wherever |grad psi| is small while phi(1-phi) is not (white noise,
grains collapsing below a few cells): there a rounding difference of two
correct implementations grows until it saturates at the size of phi(1-phi).
Long parity runs therefore use ideal-profile fields (a tilted periodic slab,
an isolated grain), on which |grad psi| = 1; noisy fields are compared over a
few steps only.
"""
import numpy as np

import oracle


def slab111(lam=1.5):
    """(45, 30, 90) box, periodic slab with normal (1,1,1): P = 15/sqrt(3) dx.
    Ragged against the 64 x 4 x 32 tiles along every axis."""
    return oracle.init_planar((45, 30, 90), (1, 1, 1), 0.37, lam=lam)


def sphere12(lam=2.0):
    """(45, 37, 70) box with one grain of radius 12 dx off the grid points."""
    return oracle.init_spheres((45, 37, 70), [(34.7, 18.3, 22.1)], [12.0], lam=lam)


def noisy_field(shape, lam, seed):
    """A [100] slab and a grain with a small seeded perturbation, clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    slab = oracle.init_planar(shape, (1, 0, 0), 0.37, lam=lam)
    sph = oracle.init_spheres(shape, [(0.3 * nx, 0.5 * ny, 0.4 * nz)], [0.3 * min(shape)], lam=lam)
    phi = 1 - (1 - slab) * (1 - sph) + 0.01 * (rng.random(shape) - 0.5)
    return np.clip(phi, 0.0, 1.0)


def as_f32_input(phi):
    """The FP32 runs and the oracle start from the same FP32-rounded values."""
    return phi.astype(np.float32).astype(np.float64)


def stable_dt(p, cap=0.1):
    """dt = min(cap, 0.8 x the explicit stability bound) for oracle parameters p."""
    return min(cap, 0.8 * oracle.stable_dt(p))
