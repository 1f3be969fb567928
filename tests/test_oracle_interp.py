"""Pins of the interpolation functions of Tab. 2 (h3, h5, h_Abel) in the oracle,
and of the model comparison of Sec. 3.1 / Fig. 7 that they enter."""
import math

import numpy as np
import pytest

import oracle

INTERPS = ("h3", "h5", "habel")


@pytest.mark.parametrize("which", INTERPS)
def test_interp_endpoints_and_symmetry(which):
    assert oracle.interp(which, 0.0) == 0.0 and oracle.interp(which, 1.0) == 1.0
    for phi in np.linspace(0.0, 1.0, 41):
        assert abs(oracle.interp(which, phi) + oracle.interp(which, 1.0 - phi) - 1.0) < 1e-15
        assert oracle.interp_prime(which, phi) >= 0.0


@pytest.mark.parametrize("which", INTERPS)
def test_interp_prime_is_the_derivative(which):
    h = 1e-5
    for phi in np.linspace(0.02, 0.98, 49):
        fd = (oracle.interp(which, phi + h) - oracle.interp(which, phi - h)) / (2 * h)
        assert abs(fd - oracle.interp_prime(which, phi)) < 1e-8


def test_interp_closed_forms_in_x():
    """h3' = 6x, h5' = 30x^2, h_Abel' = 2x/(1-2x)^2 with x = phi(1-phi)."""
    for phi in np.linspace(0.0, 1.0, 21):
        x = phi * (1 - phi)
        assert oracle.interp_prime("h3", phi) == pytest.approx(6 * x, abs=1e-15)
        assert oracle.interp_prime("h5", phi) == pytest.approx(30 * x * x, abs=1e-15)
        assert oracle.interp_prime("habel", phi) == pytest.approx(2 * x / (1 - 2 * x) ** 2, abs=1e-14)


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("which", ["h5", "habel"])
@pytest.mark.parametrize("coupling", ["cf", "global"])
def test_gradient_flow_with_each_interp(which, coupling):
    """Eq. 2 stays the gradient flow of Eq. 1 with mu h(phi) for every h."""
    rng = np.random.default_rng(5)
    shape = (6, 7, 8)
    phi = np.clip(oracle.front(shape, unit([1, 2, 2]), 0.0, lam=2.5) + 0.1 * rng.random(shape), 0, 1)
    p = oracle.params(shape, lam=2.5, mu=0.07, M=1.3, Gamma=0.8, stencil=26, coupling=coupling,
                      u=tuple(unit([1, 2, 0])), dx=0.7, interp=which)
    r = oracle.rate(p, phi)
    h = 1e-5
    dF = (oracle.energy(p, phi + h * r, True) - oracle.energy(p, phi - h * r, True)) / (2 * h)
    expect = -(3 * p.lam * p.Gamma / (2 * p.M)) * p.dx ** 3 * np.sum(r * r)
    assert abs(dF / expect - 1) < 1e-6


def bulk_rate_near_one(interp, lam, mu, delta=1e-7):
    """d(1 - phi)/dt / (1 - phi) for the uniform state phi = 1 - delta (CF)."""
    shape = (3, 3, 3)
    p = oracle.params(shape, lam=lam, mu=mu, stencil=26, coupling="cf", interp=interp)
    r = oracle.rate(p, np.full(shape, 1.0 - delta))
    return -r[1, 1, 1] / delta


@pytest.mark.parametrize("lam", [0.5, 1.0, 2.5, 4.0])
def test_cf_h3_phase_stability_limit(lam):
    """Sec. 3.1: CF + h3 keeps the unfavoured phase metastable only for
    |mu~| < 8 / (3 C_Gamma lambda~), C_Gamma = 2/3 for CF."""
    limit = 8.0 / (3.0 * (2.0 / 3.0) * lam)
    assert bulk_rate_near_one("h3", lam, 0.98 * limit) < 0
    assert bulk_rate_near_one("h3", lam, 1.02 * limit) > 0


def test_cf_h5_is_stable_for_any_driving_force():
    """Sec. 3.1: CF + h5 keeps phase stability for arbitrarily large driving forces."""
    for lam in (0.5, 2.5, 4.0):
        for mu in (1.0, 10.0, 1000.0):
            assert bulk_rate_near_one("h5", lam, mu) < 0


def slab_velocity(coupling, interp, lam, mu, dt=0.05, n=64, warm=4000, steps=8000):
    """[100] slab of period n dx (two interfaces), 6 neighbours: the mean outward
    interface velocity over the window."""
    shape = (3, 3, n)
    p = oracle.params(shape, lam=lam, mu=mu, stencil=6, coupling=coupling, dt=dt, interp=interp)
    phi = oracle.step(p, oracle.init_planar(shape, (1, 0, 0), 0.37, lam=lam), warm)
    v0 = math.fsum(phi.ravel())
    phi = oracle.step(p, phi, steps)
    return (math.fsum(phi.ravel()) - v0) / (2 * 9) / (steps * dt)


@pytest.mark.parametrize("interp", INTERPS)
def test_cf_models_pin_at_low_resolution(interp):
    """Fig. 7: every CF model is pinned at lambda~ = 2.5 for mu~ < 0.02."""
    assert abs(slab_velocity("cf", interp, 2.5, 0.01)) < 1e-7


def test_ti_moves_where_cf_pins():
    v = slab_velocity("local", "h3", 2.5, 0.01)
    assert abs(v / -0.01 - 1.0) < 1e-4


@pytest.mark.parametrize("interp", INTERPS)
def test_cf_friction_at_lambda_4(interp):
    """Fig. 7: at lambda~ = 4 the CF models run with a nearly constant relative
    velocity error of about 2e-2 at small driving forces (grid friction)."""
    err = slab_velocity("cf", interp, 4.0, 0.01) / -0.01 - 1.0
    assert -4e-2 < err < -1e-2
