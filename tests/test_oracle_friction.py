"""Pins of the grid friction force study (Fig. 3) in the oracle: the total
force on an ideal planar front, the system sum of the bracket of Eq. 4,
sampled while the front is translated through the grid.  The 300 x 1 x 1
system of the paper is a line of points between contact-angle walls that hold
the exact ideal profile (Eq. 7 with sin(alpha) = n . e), so every stencil
neighbour off the line sees the analytic front."""
import math

import numpy as np
import pytest

import oracle

U120 = (1 / math.sqrt(5), 2 / math.sqrt(5), 0.0)


def front_force(coupling, lam, n, c, u=(1.0, 0.0, 0.0), stencil=26):
    shape = (1, 1, 300)
    p = oracle.params(shape, lam=lam, stencil=stencil, coupling=coupling, u=u, mu=0.0)
    phi = oracle.front(shape, n, c, lam=lam)
    rate = oracle.rate_walls(p, phi, 7, oracle.front_sin_alpha(n))
    return math.fsum(rate.ravel()) / (2 * p.M / (3 * p.C_Gamma * lam * lam))


def amplitude(coupling, lam, n, u=(1.0, 0.0, 0.0), K=12):
    F = [front_force(coupling, lam, n, c, u) for c in np.arange(K) / K]
    return 0.5 * (max(F) - min(F)), max(abs(f) for f in F)


def rot001(deg):
    t = math.radians(deg)
    return (math.cos(t), math.sin(t), 0.0)


def rot011(deg):
    t = math.radians(deg)
    return (math.cos(t), math.sin(t) / math.sqrt(2), math.sin(t) / math.sqrt(2))


@pytest.mark.parametrize("lam", [1.0, 3.0])
@pytest.mark.parametrize("n", [rot001(0), rot001(20), rot011(35), rot001(63.43494882)])
def test_ti_n_front_feels_no_grid_force(lam, n):
    """TI_n restores translational invariance along the local normal: the
    ideal front is in discrete equilibrium at every position."""
    assert amplitude("local", lam, n)[1] < 1e-9


def test_ti_120_is_free_only_along_120():
    theta = math.degrees(math.atan(2.0))
    assert amplitude("global", 1.0, rot001(theta), U120)[1] < 1e-12
    assert amplitude("global", 1.0, rot001(0), U120)[0] > 1e-2


def test_cf_force_is_order_one_at_lambda_1_and_small_at_3():
    """Fig. 3: CF oscillations reach order unity at lambda~ = 1 and drop by
    orders of magnitude at lambda~ = 3."""
    a1 = amplitude("cf", 1.0, rot001(0))[0]
    a3 = amplitude("cf", 3.0, rot001(0))[0]
    assert 0.3 < a1 < 3.0
    assert a3 < 1e-2 * a1


def test_cf_force_decreases_towards_the_diagonal():
    amps = [amplitude("cf", 3.0, rot001(d))[0] for d in (0, 15, 30, 45)]
    assert all(b < a for a, b in zip(amps, amps[1:]))


def test_force_oscillates_with_the_lattice_period():
    """A [100] front moved by one grid spacing sees the same force."""
    for c in (0.1, 0.37, 0.8):
        assert abs(front_force("cf", 1.0, rot001(0), c) - front_force("cf", 1.0, rot001(0), c + 1.0)) < 1e-12
