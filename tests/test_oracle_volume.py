"""Pins of the oracle's constant-volume stepping, box particle and contour
statistics (Sec. 3.3), against facts that do not come from the oracle:
exact volume conservation, the Gibbs-Thomson equilibrium of a sphere
(mu = -Gamma kappa, kappa = 2/R, the sharp-interface limit of Eq. 2 whose
planar form v = -M mu / Gamma is Sec. 2.1), linearity of psi on an ideal
planar front, and the 1/(8R) curvature error of edge interpolation."""
import math

import numpy as np
import pytest

import oracle


def sphere_case(R, lam, n, Gamma=1.0, M=1.0):
    shape = (n, n, n)
    c = (n / 2 + 0.3, n / 2 - 0.2, n / 2 + 0.1)
    phi = oracle.init_spheres(shape, [c], [R], lam=lam)
    p = oracle.params(shape, lam=lam, stencil=26, coupling="local", dt=0.1, Gamma=Gamma, M=M)
    return p, phi


def test_constant_volume_conserves_the_sum():
    p, phi = sphere_case(10.0, 3.0, 32)
    v0 = math.fsum(phi.ravel())
    out, mu = oracle.step_constant_volume(p, phi, 150)
    assert abs(math.fsum(out.ravel()) - v0) <= 1e-13 * v0
    assert np.all(mu < 0)                     # a phase-1 sphere needs mu < 0 to stay


@pytest.mark.parametrize("R,lam,n", [(12.0, 3.0, 40), (16.0, 3.0, 48), (12.0, 2.0, 40)])
def test_constant_volume_mu_is_gibbs_thomson(R, lam, n):
    p, phi = sphere_case(R, lam, n)
    out, mu = oracle.step_constant_volume(p, phi, 300)
    RV = oracle.sphere_radius_from_volume(math.fsum(out.ravel()), lam)
    assert abs(mu[-1] / (-2.0 * p.Gamma / RV) - 1.0) < 1e-2
    assert abs(mu[-1] - mu[-50]) < 1e-3 * abs(mu[-1])      # settled


def test_gibbs_thomson_scales_with_gamma():
    p1, phi = sphere_case(12.0, 3.0, 40, Gamma=1.0)
    p2, _ = sphere_case(12.0, 3.0, 40, Gamma=2.0)
    _, mu1 = oracle.step_constant_volume(p1, phi, 200)
    _, mu2 = oracle.step_constant_volume(p2, phi, 200)
    assert abs(mu2[-1] / mu1[-1] - 2.0) < 1e-9


def test_contour_points_lie_on_a_tilted_planar_front():
    """psi is linear along every edge of an ideal planar front, so the l = 1/2
    points are exact (edges that wrap across the box are left out)."""
    shape, lam = (10, 12, 30), 2.5
    n = np.array([1.0, 0.35, -0.2])
    n /= np.linalg.norm(n)
    phi = oracle.front(shape, n, 0.4, lam=lam)
    p = oracle.params(shape, lam=lam)
    pts = oracle.contour_points(p, phi)
    inner = pts[(pts[:, 0] < shape[2] - 1) & (pts[:, 1] < shape[1] - 1) & (pts[:, 2] < shape[0] - 1)]
    c = 0.5 * (shape[2] * n[0] + shape[1] * n[1] + shape[0] * n[2]) + 0.4
    assert inner.shape[0] > 100
    assert np.abs(inner @ n - c).max() < 1e-12


@pytest.mark.parametrize("R", [12.0, 16.0])
def test_sphericity_of_the_ideal_sphere(R):
    """On the ideal radial profile psi = r - R exactly; along an edge r is convex
    with r'' <= 1/r, so each point errs by at most 1/(8R) inwards."""
    p, phi = sphere_case(R, 3.0, int(2 * R + 16))
    eps, Rm, Rmin, Rmax, c, npts = oracle.sphericity(p, phi)
    assert npts > 1000
    assert 0.0 < eps < 1.0 / (8.0 * R * R)
    n = phi.shape[0]
    off = np.abs(c - np.array([n / 2 + 0.3, n / 2 - 0.2, n / 2 + 0.1])).max()
    assert off < 1e-3                      # barycentre: the tails' periodic images move it slightly
    assert R - 1.0 / (8.0 * R) - 2 * off <= Rmin and Rmax <= R + 2 * off


def test_sphericity_error_scales_as_one_over_r_squared():
    e12 = oracle.sphericity(*sphere_case(12.0, 3.0, 40))[0]
    e16 = oracle.sphericity(*sphere_case(16.0, 3.0, 48))[0]
    assert abs(e12 / e16 / (16.0 / 12.0) ** 2 - 1.0) < 0.1


def test_box_particle_faces():
    """The phi = 1/2 contour crosses the axes through the box centre at the faces."""
    shape, lam = (40, 40, 40), 3.0
    lo, hi = (8.3, 10.0, 9.6), (31.3, 29.0, 30.6)
    phi = oracle.init_box(shape, lo, hi, lam=lam)
    p = oracle.params(shape, lam=lam)
    pts = oracle.contour_points(p, phi)
    for d in range(3):
        others = [a for a in range(3) if a != d]
        mid = [(lo[a] + hi[a]) / 2 for a in others]
        on_axis = pts[(np.abs(pts[:, others[0]] - round(mid[0])) < 1e-9) &
                      (np.abs(pts[:, others[1]] - round(mid[1])) < 1e-9)]
        got = sorted(on_axis[:, d])
        assert len(got) == 2
        assert abs(got[0] - lo[d]) < 1e-3 and abs(got[1] - hi[d]) < 1e-3


def _linear_psi_field(shape, n, c0):
    """phi = 1 / (1 + e^s) with s = n.x - c0: psi = ln((1-phi)/phi) = s is
    linear, so trilinear interpolation reproduces it exactly."""
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = n[0] * xx + n[1] * yy + n[2] * zz - c0
    return 1.0 / (1.0 + np.exp(s))


def test_ray_radii_exact_for_a_linear_psi():
    """Where psi is linear (an ideal planar front) the ray meets psi = 0 at
    t = (c0 - n.centre) / (n.d) exactly; the oracle finds it to the bisection
    tolerance."""
    shape = (40, 40, 40)
    n = np.array([1.0, 0.4, -0.3])
    n /= np.linalg.norm(n)
    centre = np.array([20.3, 19.7, 20.1])
    c0 = float(n @ centre) + 9.3
    phi = _linear_psi_field(shape, n, c0)
    rng = np.random.default_rng(5)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d = d[d @ n >= 0.55][:100]     # crossings within 17 cells: no wrap before them
    r = oracle.ray_radii(phi, centre, d)
    exact = (c0 - n @ centre) / (d @ n)
    assert np.all(np.abs(r - exact) < 1e-9)


def test_ray_radii_of_an_ideal_grain():
    """For the ideal radial profile psi is linear in r = |x - c| but not in x:
    trilinear interpolation errs by at most (3/8) max|d2 r| = 3 / (8 R) over a
    unit cell, and only inwards (r is convex).  A ray from outside the grain
    gives NaN."""
    shape, R, cen = (40, 40, 40), 12.0, (19.6, 20.2, 20.1)
    phi = oracle.init_spheres(shape, [cen], [R], lam=3.0)
    rng = np.random.default_rng(9)
    d = rng.normal(size=(300, 3))
    r = oracle.ray_radii(phi, cen, d)
    assert np.all(r <= R + 1e-9) and np.all(r >= R - 3.0 / (8.0 * R))
    assert np.isnan(oracle.ray_radii(phi, (2.0, 2.0, 2.0), d[:5])).all()
