"""Pins of the oracle's crop helpers, which the full-size parity tests use to
compute sampled reference values one point at a time.

* ``spheres_at`` must give the field of ``init_spheres`` at any grid point of the
  box (grains across the periodic faces included).
* ``cone_step`` must give the value of a full periodic step run at each point.
  It relies on the locality of the explicit step of Eq. 2: after K steps a
  point depends only on the (2K+1)^3 box around it (26 neighbours reach one
  cell per step, and the TI_n normal uses face neighbours only).  The full-box
  run is the independent reference here; a wrong crop axis, wrap or centre
  fails it because the box and the field have no symmetry.
"""
import numpy as np
import pytest

import oracle


def grains_box(shape, seed):
    """A few grains in a non-cubic periodic box, two of them across its faces."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    centers = [(0.4, ny * 0.55, nz * 0.3), (nx * 0.6, ny - 0.7, nz * 0.8),
               (nx * 0.5, ny * 0.25, 0.2)]
    radii = [3.2, 2.7, 2.1]
    centers = [tuple(c + rng.uniform(-0.3, 0.3) for c in cc) for cc in centers]
    return centers, radii


@pytest.mark.parametrize("shape", [(13, 11, 16), (9, 17, 10)])
def test_spheres_at_equals_init_spheres(shape):
    nz, ny, nx = shape
    centers, radii = grains_box(shape, 7)
    full = oracle.init_spheres(shape, centers, radii, lam=2.5)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=-1)
    got = oracle.spheres_at(shape, centers, radii, xyz, lam=2.5).reshape(shape)
    np.testing.assert_array_equal(got, full)
    # interface values exist on both sides of the periodic faces (the test is not vacuous)
    band = (full > 1e-3) & (full < 1 - 1e-3)
    assert band[0].any() and band[-1].any() and band[:, :, 0].any() and band[:, :, -1].any()


@pytest.mark.parametrize("coupling,stencil,steps", [("local", 26, 3), ("global", 18, 2),
                                                    ("cf", 6, 4), ("local", 6, 1), ("local", 26, 0)])
def test_cone_step_equals_full_periodic_step(coupling, stencil, steps):
    shape = (13, 11, 16)
    nz, ny, nx = shape
    centers, radii = grains_box(shape, 11)
    lam = 2.5
    phi0 = oracle.init_spheres(shape, centers, radii, lam=lam)
    p_full = oracle.params(shape, lam=lam, mu=0.03, dt=0.05, stencil=stencil, coupling=coupling,
                           u=(1.0, 2.0, 0.0))
    full = oracle.step(p_full, phi0.copy(), steps)
    rng = np.random.default_rng(3)
    # every corner and face neighbourhood (cones that wrap on one, two or three
    # axes), plus random points
    pts = [(x, y, z) for x in (0, 1, nx - 1) for y in (0, ny - 2) for z in (0, nz - 1)]
    pts += [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(20)]
    field_at = lambda xyz: phi0[xyz[:, 2], xyz[:, 1], xyz[:, 0]]
    p_crop = oracle.params((3, 3, 3), lam=lam, mu=0.03, dt=0.05, stencil=stencil, coupling=coupling,
                           u=(1.0, 2.0, 0.0))
    got = oracle.cone_step(p_crop, shape, field_at, pts, steps)
    want = np.array([full[z, y, x] for (x, y, z) in pts])
    np.testing.assert_array_equal(got, want)
    if steps > 0:   # the steps moved the field at the sampled points
        assert np.max(np.abs(want - np.array([phi0[z, y, x] for (x, y, z) in pts]))) > 1e-6


def test_cone_step_with_spheres_at_equals_full_grain_run():
    """The composition the full-size tests use: crops built by spheres_at."""
    shape = (12, 14, 15)
    nz, ny, nx = shape
    centers, radii = grains_box(shape, 5)
    lam = 3.0
    phi0 = oracle.init_spheres(shape, centers, radii, lam=lam)
    p = oracle.params(shape, lam=lam, mu=0.01, dt=0.1, stencil=26, coupling="local")
    full = oracle.step(p, phi0.copy(), 4)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (7, 3, 11), (14, 13, 5), (2, 9, 0)]
    field_at = lambda xyz: oracle.spheres_at(shape, centers, radii, xyz, lam=lam)
    pc = oracle.params((3, 3, 3), lam=lam, mu=0.01, dt=0.1, stencil=26, coupling="local")
    got = oracle.cone_step(pc, shape, field_at, pts, 4)
    np.testing.assert_array_equal(got, [full[z, y, x] for (x, y, z) in pts])
