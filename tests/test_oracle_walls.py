"""Pins of the oracle's contact-angle walls (Sec. 2.2, Eq. 7) against facts
that do not come from the oracle: the tanh addition law, the analytic tilted
front of Eq. 3, the stationarity of a translationally invariant model on its
ideal profile, and the kinetics v_n = -M mu / Gamma of Sec. 2.1."""
import math

import numpy as np
import pytest

import oracle


def ideal(s, lam):
    return 0.5 * (1.0 - np.tanh(2.0 * np.asarray(s, dtype=np.float64) / lam))


def rot001(theta):
    return (math.cos(theta), math.sin(theta), 0.0)


def rot011(theta):
    return (math.cos(theta), math.sin(theta) / math.sqrt(2.0), math.sin(theta) / math.sqrt(2.0))


@pytest.mark.parametrize("lam", [0.7, 2.0, 4.0])
def test_wall_value_is_the_shifted_ideal_profile(lam):
    """Eq. 7 moves a value along the ideal profile by the length delta with
    tanh(2 delta / lambda) = a."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        s = rng.uniform(-3 * lam, 3 * lam)
        d = rng.uniform(-1.5, 1.5)
        a, f = math.tanh(2.0 * d / lam), ideal(s, lam)
        got = oracle.wall_value(f, a)
        # the input's rounding (1 ulp) is carried with the map's slope (1 - a^2)/den^2
        slope = (1.0 - a * a) / (1.0 - a * (2.0 * f - 1.0)) ** 2
        assert abs(got - ideal(s + d, lam)) < 3e-16 * (1.0 + slope)
    for a in (-0.9, -0.2, 0.0, 0.5, 0.99):
        assert oracle.wall_value(0.0, a) == 0.0 and oracle.wall_value(1.0, a) == 1.0


def analytic_front_padded(shape, walls, n, offset, lam, dx=1.0):
    """Eq. 3 for the front at every padded point, interior index i at padded i + g."""
    nz, ny, nx = shape
    gz, gy, gx = (walls >> 2) & 1, (walls >> 1) & 1, walls & 1
    v = np.asarray(n, dtype=np.float64) / np.linalg.norm(n)
    Z, Y, X = np.meshgrid(np.arange(nz + 2 * gz) - gz, np.arange(ny + 2 * gy) - gy,
                          np.arange(nx + 2 * gx) - gx, indexing="ij")
    c = 0.5 * dx * (nx * v[0] + ny * v[1] + nz * v[2]) + offset
    return ideal(dx * (X * v[0] + Y * v[1] + Z * v[2]) - c, lam)


@pytest.mark.parametrize("n", [rot001(0.4), rot011(0.7), (1.0, 0.4, -0.3), (0.2, -1.0, 0.5)])
@pytest.mark.parametrize("walls", [7, 6, 3])
def test_fill_reproduces_the_tilted_front(n, walls):
    """Faces, edges and corners: every ghost equals the analytic front."""
    shape, lam = (7, 6, 9), 2.5
    p = oracle.params(shape, lam=lam)
    exact = analytic_front_padded(shape, walls, n, 0.31, lam)
    phi = oracle.pad(oracle.front(shape, n, 0.31, lam=lam), walls)
    assert np.abs(oracle.interior(phi, walls) - oracle.interior(exact, walls)).max() < 1e-15
    oracle.fill_walls(p, phi, walls, oracle.front_sin_alpha(n))
    assert np.abs(phi - exact).max() < 1e-14


@pytest.mark.parametrize("stencil", [6, 18, 26])
@pytest.mark.parametrize("coupling", ["global", "local"])
@pytest.mark.parametrize("n", [rot001(0.35), rot011(0.6), (1.0, 0.45, -0.3)])
def test_walled_front_is_stationary(stencil, coupling, n):
    """TI with u = n (and TI_n) holds the ideal tilted front exactly at mu = 0,
    also next to the walls and their edges; flipping the walls' angles breaks it."""
    shape, lam = (8, 9, 14), 3.0
    p = oracle.params(shape, lam=lam, stencil=stencil, coupling=coupling, u=n, mu=0.0)
    phi = oracle.front(shape, n, 0.2, lam=lam)
    sa = oracle.front_sin_alpha(n)
    assert np.abs(oracle.rate_walls(p, phi, 7, sa)).max() < 1e-12
    wrong = [-v for v in sa]
    assert np.abs(oracle.rate_walls(p, phi, 7, wrong)).max() > 1e-3


def test_cf_front_is_not_stationary():
    """Control: the continuum-field potential is not translationally invariant."""
    shape, lam, n = (8, 9, 14), 3.0, rot001(0.35)
    p = oracle.params(shape, lam=lam, stencil=26, coupling="cf", mu=0.0)
    phi = oracle.front(shape, n, 0.2, lam=lam)
    assert np.abs(oracle.rate_walls(p, phi, 7, oracle.front_sin_alpha(n))).max() > 1e-4


@pytest.mark.parametrize("axis,theta", [("001", 0.45), ("011", 0.6)])
def test_tilted_front_moves_at_the_kinetic_velocity(axis, theta):
    """Sec. 3.2 set-up on a small box: with mu = mu0 cos(theta) the front's
    x-velocity is -M mu0 / Gamma for every orientation (TI_n, 26 neighbours)."""
    n = rot001(theta) if axis == "001" else rot011(theta)
    shape, lam, mu0, dt = (6, 6, 24), 4.0, 0.05, 0.05
    mu = mu0 * math.cos(theta)
    p = oracle.params(shape, lam=lam, stencil=26, coupling="local", mu=mu, dt=dt)
    sa = oracle.front_sin_alpha(n)
    phi = oracle.step_walls(p, oracle.front(shape, n, -2.0, lam=lam), 7, sa, 200)
    v0 = math.fsum(phi.ravel())
    steps = 600
    phi = oracle.step_walls(p, phi, 7, sa, steps)
    v1 = math.fsum(phi.ravel())
    vx = (v1 - v0) / (shape[0] * shape[1]) / (steps * dt)
    assert abs(vx / (-mu0) - 1.0) < 3e-3, vx
