"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the printed
Tab. 1, closed forms derived from Eq. 3-6, the independent 1D brute force,
exact invariances, energy identities and the paper's qualitative claims.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle1d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ideal_field(shape, n, c, lam, dx=1.0):
    """Eq. 3 sampled directly (phi decreasing along n)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = dx * (x * n[0] + y * n[1] + z * n[2])
    return 0.5 * (1.0 - np.tanh(2.0 * (s - c) / lam))


def unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------- P1 ---
def read_tab1():
    rows = []
    with open(os.path.join(GOLDEN, "tab1_directions.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, sh, r, mr, dot, col = line.split()
            rows.append((int(k), int(sh), tuple(map(int, r.split(","))),
                         tuple(map(int, mr.split(","))), int(dot), int(col)))
    return rows


def test_directions_match_tab1(orc):
    rows = read_tab1()
    assert len(rows) == 13
    for k, sh, r, mr, dot, col in rows:
        rk, shell = orc.direction(k)
        assert shell == sh
        assert rk in (r, mr) and tuple(-v for v in rk) in (r, mr)
        assert sum(v * v for v in rk) == sh          # |r_k| = sqrt(j) dx
        # printed dot product with [120], up to the sign of the representative
        assert abs(np.dot(rk, (1, 2, 0))) == abs(dot)


def test_tab1_last_column_is_eq5_per_shell(orc):
    """|arctanh a_k| = 2 |r_k.u| / lambda (Eq. 5); the printed column agrees
    per shell as a multiset (the only thing that enters the sums)."""
    rows = read_tab1()
    for sh in (1, 2, 3):
        printed = sorted(col for k, s, r, mr, dot, col in rows if s == sh)
        eq5 = sorted(2 * abs(int(np.dot(orc.direction(k)[0], (1, 2, 0))))
                     for k, s, *_ in rows if s == sh)
        assert printed == eq5


def test_nu_makes_each_shell_a_laplacian(orc):
    """nu_j sum_{k in j} e_k e_k^T = I for nu_j = 3/m_j (Sec. 2.1)."""
    for sh, ks in ((1, range(0, 3)), (2, range(3, 9)), (3, range(9, 13))):
        T = np.zeros((3, 3))
        for k in ks:
            r = np.array(orc.direction(k)[0], dtype=float)
            e = r / np.linalg.norm(r)
            T += np.outer(e, e)
        np.testing.assert_allclose(orc.nu(sh) * T, np.eye(3), atol=1e-15)


# --------------------------------------------------------------------- P2 ---
@pytest.mark.parametrize("a", [0.05, 0.3, 0.6, 0.9, 0.999])
def test_potential_endpoints_and_derivative(orc, a):
    rho, lam = math.sqrt(2.0), 1.7
    assert orc.g(0.0, a, rho, lam) == 0.0 and orc.g(1.0, a, rho, lam) == 0.0
    for phi in np.linspace(0.01, 0.99, 23):
        h = 1e-6
        fd = (orc.g(phi + h, a, rho, lam) - orc.g(phi - h, a, rho, lam)) / (2 * h)
        gp = orc.g_prime(phi, a, rho, lam)
        assert abs(fd - gp) < 1e-7 * max(1.0, abs(gp))
        # independent route: complex-step derivative of Eq. 6 as printed
        cs = oracle1d.g_prime_complex_step(phi, a, rho, lam)
        assert abs(cs - gp) < 1e-12 * max(1.0, abs(gp))


def test_potential_matches_printed_eq6_where_well_conditioned(orc):
    for a in (0.3, 0.5, 0.8):
        for phi in np.linspace(0.02, 0.98, 17):
            printed = float(oracle1d.g_eq6(phi, a, 1.0, 2.0))
            assert abs(orc.g(phi, a, 1.0, 2.0) - printed) < 1e-13


def test_potential_small_coupling_is_stable(orc):
    """For a -> 0, g -> (lambda/r)^2 * 2 a^2 x^2 (leading order of Eq. 6)."""
    for a in (1e-3, 1e-5, 1e-8):
        for phi in (0.1, 0.5, 0.77):
            x = phi * (1 - phi)
            lead = 2.0 * a * a * x * x
            assert abs(orc.g(phi, a, 1.0, 1.0) / lead - 1.0) < 10 * a * a + 1e-12


def test_potential_continuum_limit(orc):
    """lambda/dx -> infinity: sum_k gamma_j nu_j g_k -> 8 phi^2 (1-phi)^2 for any n
    (the conventional quartic double well, Sec. 2.1)."""
    lam = 4000.0
    n = unit([0.3, -0.7, 0.2])
    gam = orc.default_gamma(26)
    for phi in (0.2, 0.5, 0.9):
        s = 0.0
        for k in range(13):
            r, sh = orc.direction(k)
            rho = math.sqrt(sh)
            a = math.tanh(2.0 * np.dot(r, n) / lam)
            s += gam[sh - 1] * orc.nu(sh) * orc.g(phi, a, rho, lam)
        x = phi * (1 - phi)
        assert abs(s / (8 * x * x) - 1.0) < 1e-5


# --------------------------------------------------------------------- P3 ---
def test_ideal_second_difference_equals_potential_force(orc):
    """For Eq. 3 sampled at p and p +- r, phi+ - 2 phi + phi- = (r^2/lambda^2) g_k'(phi)
    with a_k from Eq. 5: every direction is in discrete equilibrium (Eq. 4)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        lam = rng.uniform(0.4, 6.0)
        n = unit(rng.normal(size=3))
        k = int(rng.integers(13))
        r, sh = orc.direction(k)
        rho = math.sqrt(sh)
        s0 = rng.uniform(-1.5, 1.5) * lam
        prof = lambda s: 0.5 * (1 - math.tanh(2 * s / lam))
        rn = float(np.dot(r, n))
        phi, pp, pm = prof(s0), prof(s0 + rn), prof(s0 - rn)
        a = math.tanh(2 * rn / lam)
        lhs = pp - 2 * phi + pm
        rhs = rho * rho / lam ** 2 * orc.g_prime(phi, a, rho, lam)
        assert abs(lhs - rhs) < 1e-13


# --------------------------------------------------------------------- P4 ---
@pytest.mark.parametrize("stencil", [6, 18, 26])
@pytest.mark.parametrize("coupling", ["local", "global"])
def test_one_step_rate_is_exact_travelling_wave(orc, stencil, coupling):
    """On the ideal profile, d_t phi = -(4 M mu / (lambda Gamma)) phi (1 - phi) at every
    point: the semi-discrete TI scheme moves it at v = -M mu / Gamma exactly."""
    rng = np.random.default_rng(stencil + (7 if coupling == "local" else 0))
    shape = (11, 12, 13)
    for _ in range(3):
        lam = rng.uniform(0.8, 5.0)
        n = unit(rng.normal(size=3))
        mu = rng.uniform(-0.1, 0.1)
        M, Gamma = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
        phi = ideal_field(shape, n, 6.0 + rng.uniform(), lam)
        p = orc.params(shape, lam=lam, mu=mu, M=M, Gamma=Gamma, stencil=stencil,
                       coupling=coupling, u=tuple(n), eps=1e-300)
        r = orc.rate(p, phi)
        exact = -(4 * M * mu / (lam * Gamma)) * phi * (1 - phi)
        inner = (slice(1, -1),) * 3
        assert np.abs(r - exact)[inner].max() < 2e-14


def test_cf_control_is_not_translation_invariant(orc):
    """Negative control: the CF potential leaves grid forces on the ideal profile."""
    shape = (9, 9, 30)
    phi = ideal_field(shape, (1, 0, 0), 14.3, 2.0)
    p = orc.params(shape, lam=2.0, mu=0.0, stencil=26, coupling="cf")
    r = orc.rate(p, phi)
    assert np.abs(r).max() > 1e-3


# --------------------------------------------------------------------- P5 ---
@pytest.mark.parametrize("coupling", ["local", "global"])
def test_stationary_at_zero_driving_force(orc, coupling):
    """mu = 0: the ideal profile is a fixed point of the fully discrete scheme.
    Boundary layer held at the analytic values (ghosts)."""
    shape = (10, 10, 10)
    n = unit([1.0, 2.0, 3.0])
    lam = 2.5
    phi0 = ideal_field(shape, n, 8.1, lam)
    p = orc.params(shape, lam=lam, mu=0.0, stencil=26, coupling=coupling, u=tuple(n),
                   eps=1e-300)
    phi = phi0.copy()
    edge = np.ones(shape, bool)
    edge[1:-1, 1:-1, 1:-1] = False
    for _ in range(100):
        phi = orc.step(p, phi, 1)
        phi[edge] = phi0[edge]
    assert np.abs(phi - phi0).max() < 1e-13


# --------------------------------------------------------------------- P6 ---
def slab_velocity_1d(orc, *, lam, mu, dt, steps, nx=160, coupling="global", stencil=6):
    shape = (1, 1, nx)
    phi = orc.init_planar(shape, (1, 0, 0), 0.3, lam=lam)
    p = orc.params(shape, lam=lam, mu=mu, dt=dt, stencil=stencil, coupling=coupling)
    A = orc.slab_area(shape, (1, 0, 0))
    burn = steps // 4
    phi = orc.step(p, phi, burn)
    V0 = orc.phase_volume(phi)
    phi = orc.step(p, phi, steps - burn)
    V1 = orc.phase_volume(phi)
    return (V1 - V0) / A / ((steps - burn) * dt)


def test_velocity_linear_in_mu_with_euler_error(orc):
    """v = -M mu / Gamma (Sec. 2.1, energy conservation); the fully discrete scheme
    errs only by forward Euler: first order in dt, extrapolating to v_th."""
    lam, mu = 4.0, 0.08
    v1 = slab_velocity_1d(orc, lam=lam, mu=mu, dt=0.2, steps=800)
    v2 = slab_velocity_1d(orc, lam=lam, mu=mu, dt=0.1, steps=1600)
    v4 = slab_velocity_1d(orc, lam=lam, mu=mu, dt=0.05, steps=3200)
    vth = -mu
    e1, e2, e4 = v1 - vth, v2 - vth, v4 - vth
    assert abs(e2 / vth) < 1e-3
    assert 1.7 < e1 / e2 < 2.3 and 1.7 < e2 / e4 < 2.3      # first order in dt
    rich = 2 * v4 - v2                                       # Richardson
    assert abs(rich / vth - 1) < abs(e4 / vth) / 5


def contour_position_1d(phi_line, lam):
    """Position of the first phi = 1/2 crossing with phi decreasing along x, by the
    nonlinear interpolation of Eq. 8-10 at l = 1/2: the linear zero of
    psi = (lambda/4) ln((1-phi)/phi) between the two grid points."""
    with np.errstate(divide="ignore"):
        psi = 0.25 * lam * np.log((1 - phi_line) / phi_line)
    i = int(np.nonzero((psi[:-1] < 0) & (psi[1:] >= 0))[0][0])
    return i + (-psi[i]) / (psi[i + 1] - psi[i])


def test_contour_interpolation_exact_on_ideal_profile():
    for lam in (0.5, 1.0, 4.0):
        for c in (10.0, 10.37, 10.99):
            phi = oracle1d.ideal_profile(np.arange(24.0), c, lam)
            assert abs(contour_position_1d(phi, lam) - c) < 1e-12


@pytest.mark.parametrize("mu", [1e-4, -3e-3, 0.03])
def test_no_pinning_threshold(orc, mu):
    """TI at lambda = 1.5 dx moves at v_th even for tiny driving forces (Fig. 7)."""
    nx, lam, dt = 60, 1.5, 0.02
    shape = (1, 1, nx)
    phi = orc.init_planar(shape, (1, 0, 0), 0.3, lam=lam)
    p = orc.params(shape, lam=lam, mu=mu, dt=dt, stencil=6, coupling="global")
    phi = orc.step(p, phi, 500)
    c0 = contour_position_1d(phi[0, 0], lam)
    phi = orc.step(p, phi, 1500)
    v = (contour_position_1d(phi[0, 0], lam) - c0) / (1500 * dt)
    # the right-hand interface of the slab moves along +x at v_th = -M mu / Gamma
    assert abs(v / (-mu) - 1) < 1e-3


# --------------------------------------------------------------------- P7 ---
def test_cf_pins_at_small_width_while_ti_moves(orc):
    """CF + h3 at lambda = 1 dx and mu~ = 0.02 does not move; TI does (Sec. 3.1)."""
    v_cf = slab_velocity_1d(orc, lam=1.0, mu=0.02, dt=0.02, steps=3000, nx=40, coupling="cf")
    v_ti = slab_velocity_1d(orc, lam=1.0, mu=0.02, dt=0.02, steps=3000, nx=40)
    assert abs(v_cf) < 0.05 * 0.02
    assert abs(v_ti / -0.02 - 1) < 1e-2


# --------------------------------------------------------------------- P8 ---
@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
def test_cubic_symmetry(orc, coupling):
    """Permuting or reflecting the axes of the input permutes the output."""
    rng = np.random.default_rng(11)
    shape = (9, 9, 9)
    phi = ideal_field(shape, unit([0.2, 0.5, 0.9]), 4.0, 2.0) + 0.05 * rng.random(shape)
    phi = np.clip(phi, 0.0, 1.0)
    u = (0.0, 0.0, 1.0)
    p = orc.params(shape, lam=2.0, mu=0.02, stencil=26, coupling=coupling, u=u)
    r = orc.rate(p, phi)
    # swap x and y (u along z is invariant)
    phit = np.ascontiguousarray(np.swapaxes(phi, 1, 2))
    rt = orc.rate(p, phit)
    np.testing.assert_allclose(rt, np.swapaxes(r, 1, 2), atol=1e-14)
    # reflect x (periodic reflection x -> -x)
    phir = np.ascontiguousarray(np.roll(phi[:, :, ::-1], 1, axis=2))
    rr = orc.rate(p, phir)
    np.testing.assert_allclose(rr, np.roll(r[:, :, ::-1], 1, axis=2), atol=1e-14)


@pytest.mark.parametrize("hkl,L,lam", [((1, 1, 0), 30, 2.5), ((1, 1, 1), 36, 2.5),
                                       ((1, 2, 3), 60, 2.0)])
def test_local_velocity_independent_of_orientation(orc, hkl, L, lam):
    """TI_n: the same v for any slab orientation (Sec. 3.2, Fig. 8).  Boxes are
    sized so that each slab is at least 4 lambda thick (no tail interaction)."""
    mu, dt = 0.1, 0.05
    shape = (L, L, L)
    phi = orc.init_planar(shape, hkl, 0.4, lam=lam)
    p = orc.params(shape, lam=lam, mu=mu, dt=dt, stencil=26, coupling="local", eps=1e-300)
    A = orc.slab_area(shape, hkl)
    phi = orc.step(p, phi, 20)
    V0 = orc.phase_volume(phi)
    phi = orc.step(p, phi, 60)
    v = (orc.phase_volume(phi) - V0) / A / (60 * dt)
    assert abs(v / -mu - 1) < 1e-3


# --------------------------------------------------------------------- P9 ---
@pytest.mark.parametrize("stencil", [6, 18, 26])
@pytest.mark.parametrize("coupling", ["local", "global"])
def test_3d_oracle_equals_1d_brute_force(orc, stencil, coupling):
    nx, lam, mu = 48, 2.2, 0.04
    phi1 = oracle1d.ideal_profile(np.arange(nx), 17.37, lam) \
        + 0.02 * np.sin(2 * np.pi * np.arange(nx) / nx)
    phi3 = np.ascontiguousarray(np.broadcast_to(phi1, (3, 4, nx)))
    p = orc.params(phi3.shape, lam=lam, mu=mu, stencil=stencil, coupling=coupling,
                   eps=1e-300)
    r3 = orc.rate(p, phi3)
    r1 = oracle1d.rate(phi1, lam=lam, mu=mu, C_Gamma=p.C_Gamma)
    assert np.abs(r3 - r1).max() < 1e-14
    s3 = orc.step(p, phi3, 30)
    s1 = oracle1d.run(phi1, 30, dt=p.dt, lam=lam, mu=mu, C_Gamma=p.C_Gamma)
    assert np.abs(s3 - s1).max() < 1e-13


# ------------------------------------------------------------- energy -------
@pytest.mark.parametrize("coupling", ["global", "cf"])
@pytest.mark.parametrize("stencil", [6, 26])
def test_rate_is_gradient_flow_of_eq1(orc, coupling, stencil):
    """Eq. 2 is the gradient flow of Eq. 1: the directional derivative of F along
    the rate equals -(3 lambda Gamma / 2M) dx^3 sum rate^2."""
    rng = np.random.default_rng(3)
    shape = (7, 8, 9)
    phi = np.clip(ideal_field(shape, unit([1, 2, 2]), 5, 2.5) + 0.1 * rng.random(shape), 0, 1)
    p = orc.params(shape, lam=2.5, mu=0.03, M=1.3, Gamma=0.8, stencil=stencil,
                   coupling=coupling, u=tuple(unit([1, 2, 0])), dx=0.7)
    r = orc.rate(p, phi)
    h = 1e-5
    dF = (orc.energy(p, phi + h * r, True) - orc.energy(p, phi - h * r, True)) / (2 * h)
    expect = -(3 * p.lam * p.Gamma / (2 * p.M)) * p.dx ** 3 * np.sum(r * r)
    assert abs(dF / expect - 1) < 1e-6


def test_energy_decreases(orc):
    shape = (8, 8, 8)
    rng = np.random.default_rng(1)
    phi = rng.random(shape)
    p = orc.params(shape, lam=3.0, mu=0.0, dt=0.05, stencil=26, coupling="global")
    E = [orc.energy(p, phi)]
    for _ in range(10):
        phi = orc.step(p, phi, 1)
        E.append(orc.energy(p, phi))
    assert all(b < a for a, b in zip(E, E[1:]))


# -------------------------------------------------------------------- P12 ---
def test_ti_interface_energy_independent_of_offset(orc):
    for lam in (0.8, 1.5, 4.0):
        p = orc.params((1, 1, 100), lam=lam, stencil=6, coupling="global")
        E = [orc.energy(p, orc.init_planar((1, 1, 100), (1, 0, 0), c, lam=lam))
             for c in np.linspace(0, 1, 9)]
        assert np.ptp(E) < 1e-12
        assert abs(E[0] - 2.0) < 1e-12          # Gamma per unit area, two interfaces
    pc = orc.params((1, 1, 100), lam=1.5, stencil=6, coupling="cf")
    Ec = [orc.energy(pc, orc.init_planar((1, 1, 100), (1, 0, 0), c, lam=1.5))
          for c in np.linspace(0, 1, 9)]
    assert np.ptp(Ec) > 1e-3                   # CF energy oscillates (Fig. 1b)


def test_calibration_continuum_limit(orc):
    """C_Gamma -> 2/3 as lambda/dx -> infinity (equipartition of Eq. 1 on Eq. 3)."""
    c20, c40 = orc.calibrate_cgamma(20.0), orc.calibrate_cgamma(40.0)
    assert 3.8 < (2.0 / 3.0 - c20) / (2.0 / 3.0 - c40) < 4.2       # O((dx/lambda)^2)
    assert abs((4 * c40 - c20) / 3 - 2.0 / 3.0) < 2e-6              # Richardson
    c = [orc.calibrate_cgamma(l) for l in (0.5, 1, 2, 4, 8)]
    assert all(a < b for a, b in zip(c, c[1:])) and c[-1] < 2.0 / 3.0


# -------------------------------------------------------------------- P13 ---
@pytest.mark.parametrize("lam", [1.0, 2.0, 4.0])
def test_cf_phase_stability_limit(orc, lam):
    """CF + h3 keeps a barrier between the phases iff |mu~| < 8/(3 C_Gamma lambda~)."""
    C = 2.0 / 3.0
    lim = 8.0 / (3.0 * C * lam)

    def has_barrier(mu):
        p = orc.params((1, 1, 1), lam=lam, mu=mu, stencil=6, coupling="cf", C_Gamma=C)
        cs = np.linspace(0.001, 0.999, 999)
        r = np.array([orc.rate(p, np.full((1, 1, 1), c))[0, 0, 0] for c in cs])
        return np.any(np.diff(np.sign(r)) != 0)
    assert has_barrier(0.97 * lim) and has_barrier(-0.97 * lim)
    assert not has_barrier(1.03 * lim) and not has_barrier(-1.03 * lim)


# ------------------------------------------------------------ Laplacian -----
def mode_rate(orc, stencil, m, L=64):
    """Growth rate of a small Fourier mode about phi = 1/2 under CF (mu = 0)."""
    shape = (L, L, L) if m[2] else (1, L, L)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    th = 2 * np.pi * np.array(m) / L
    eps = 1e-7
    mode = np.cos(th[0] * x + th[1] * y + th[2] * z)
    p = orc.params(shape, lam=1.0, mu=0.0, stencil=stencil, coupling="cf", C_Gamma=2.0 / 3.0)
    r = orc.rate(p, 0.5 + eps * mode)
    # A = 2M/(3 C lambda^2) = 1; linear response = A lambda^2 sigma(theta) + 8 A
    return float(np.sum(r * mode) / np.sum(mode * mode) / eps) - 8.0, float(np.linalg.norm(th))


@pytest.mark.parametrize("stencil", [18, 26])
def test_shell_weights_give_isotropic_laplacian(orc, stencil):
    """Reading of gamma_j: 3 gamma_2 + 6 gamma_3 = 2 makes the O(dx^2) error of the
    weighted Laplacian isotropic: symbol = -|th|^2 + |th|^4/12 + O(th^6)."""
    s1, t = mode_rate(orc, stencil, (5, 0, 0))
    s2, _ = mode_rate(orc, stencil, (3, 4, 0))
    assert abs(s1 - s2) < 2e-4
    assert abs(s1 - (-t ** 2 + t ** 4 / 12)) < 2e-3


def test_six_neighbour_laplacian_is_anisotropic(orc):
    s1, _ = mode_rate(orc, 6, (5, 0, 0))
    s2, _ = mode_rate(orc, 6, (3, 4, 0))
    assert abs(s1 - s2) > 2e-3


# ------------------------------------------------------------ stability -----
def test_stable_dt_worked_values(orc):
    p6 = orc.params((4, 4, 4), lam=4.0, stencil=6, coupling="global", C_Gamma=2.0 / 3.0)
    assert abs(orc.stable_dt(p6) - 2.0 / (12.0 + 16 * 4 * math.sinh(0.5) ** 2 / 16)) < 1e-9
    p26 = orc.params((4, 4, 4), lam=3.0, stencil=26, coupling="local", C_Gamma=2.0 / 3.0)
    assert 0.2 < orc.stable_dt(p26) < 0.3


def test_stable_dt_is_sharp(orc):
    """Just above the bound a bulk perturbation grows; just below it decays."""
    shape = (4, 4, 4)
    lam = 1.0
    p = orc.params(shape, lam=lam, stencil=6, coupling="global")
    dtm = orc.stable_dt(p)
    z, y, x = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    pert = 1e-9 * (1 + (-1.0) ** (x + y + z))   # the 3D checkerboard mode
    for f, grows in ((0.97, False), (1.03, True)):
        q = orc.params(shape, lam=lam, stencil=6, coupling="global", dt=f * dtm)
        phi = orc.step(q, pert, 400)
        assert (np.abs(phi).max() > 1e-9) == grows


# -------------------------------------------------------------------- P11 ---
def test_reductions_closed_forms(orc):
    """Lattice sums of the ideal profile equal the integrals up to aliasing of
    relative size ~ (pi^2 lambda~) exp(-pi^2 lambda~ / 2) (Poisson summation)."""
    shape = (4, 4, 192)
    lam = 6.0
    phi = orc.init_planar(shape, (1, 0, 0), 0.31, lam=lam)
    V = orc.phase_volume(phi)
    assert abs(V / (phi.size / 2.0) - 1) < 1e-10
    A = orc.interface_area(phi, lam)
    assert abs(A / orc.slab_area(shape, (1, 0, 0)) - 1) < 1e-10


def test_sphere_volume_closed_form(orc):
    R, lam = 20.0, 4.0
    phi = orc.init_spheres((96, 96, 96), [(47.7, 48.2, 48.9)], [R], lam=lam)
    V = orc.phase_volume(phi)
    exact = 4 * math.pi / 3 * (R ** 3 + R * math.pi ** 2 * lam ** 2 / 16)
    assert abs(V / exact - 1) < 1e-9
    assert abs(orc.sphere_radius_from_volume(V, lam) - R) < 1e-7


def test_slab_init_periodic_and_symmetric(orc):
    for hkl, L in (((1, 2, 3), 28), ((1, 0, 0), 32), ((-2, 1, 4), 24)):
        shape = (L, L, L)
        phi = orc.init_planar(shape, hkl, 0.0, lam=2.0)
        # periodic continuation: the field is a function of p.N only
        n = unit(hkl)
        z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
        s = x * n[0] + y * n[1] + z * n[2]
        order = np.argsort(s.ravel(), kind="stable")
        sv, pv = s.ravel()[order], phi.ravel()[order]
        same = np.abs(np.diff(sv)) < 1e-9
        assert np.all(np.abs(np.diff(pv))[same] < 1e-12)
        assert abs(phi.mean() - 0.5) < 1e-3


def _ideal_sphere_radius(volume, lam):
    """R of the ideal radial profile holding `volume` of phi:
    (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16) = volume, by Newton's method."""
    k = math.pi ** 2 * lam ** 2 / 16.0
    target = 3.0 * volume / (4.0 * math.pi)
    r = target ** (1.0 / 3.0)
    for _ in range(60):
        r -= (r ** 3 + k * r - target) / (3.0 * r * r + k)
    return r


def test_grain_shrinks_by_the_curvature_law(orc):
    """P10 (approximate): at mu = 0 a grain's R^2 falls linearly in time at
    4 M sigma / Gamma with sigma = 2 Gamma / (3 C_Gamma) of the discrete model,
    up to corrections of order lambda / R.  A TI_n grain of R = 24 at lambda = 3
    over 200 steps (R ends near 22.3) must meet the law within lambda / R_end;
    a dropped shell, a wrong sign or a wrong C_Gamma scaling breaks it."""
    shape, r0, lam = (64, 64, 64), 24.0, 3.0
    phi = orc.init_spheres(shape, [(31.7, 32.2, 31.9)], [r0], lam=lam)
    p = orc.params(shape, lam=lam, mu=0.0, stencil=26, coupling="local")
    ts, radii = [0.0], [_ideal_sphere_radius(orc.phase_volume(phi), lam)]
    for i in range(2):
        phi = orc.step(p, phi, 100)
        ts.append((i + 1) * 100 * p.dt)
        radii.append(_ideal_sphere_radius(orc.phase_volume(phi), lam))
    assert abs(radii[0] - r0) < 1e-4
    rate = np.polyfit(ts, np.square(radii), 1)[0]
    law = -4.0 * p.M * (2.0 * p.Gamma / (3.0 * p.C_Gamma)) / p.Gamma
    assert abs(rate / law - 1.0) < lam / radii[-1], (rate, law)
