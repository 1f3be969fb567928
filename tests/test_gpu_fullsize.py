"""Parity at the benchmark sizes, in the launch configuration bench.py times
(FP32 tiled kernel, guided z-chunks led by 32 planes per block), on sampled
outputs.

The GPU builds its own initial field; the oracle builds its own at the
dependency cone of each sampled point (a point's value after K steps depends
only on the (2K+1)^3 box around it) and steps that crop.  The two initial
fields differ only by the FP32 rounding of the GPU's.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ZCHUNK = 32


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def sample_points(rng, shape, centers, radii, n, lam, flat=False):
    """Half uniform, half inside the interface bands of the grains (with flat,
    along directions in the x-y plane: on a grid a few planes thick a grain is
    a disc)."""
    nz, ny, nx = shape
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz)))
           for _ in range(n // 2)]
    while len(pts) < n:
        i = int(rng.integers(len(radii)))
        v = rng.normal(size=3)
        if flat:
            v[2] = 0.0
        v /= np.linalg.norm(v)
        r = radii[i] + rng.uniform(-3 * lam, 3 * lam)
        p = np.asarray(centers[i]) + r * v
        pts.append((int(round(p[0])) % nx, int(round(p[1])) % ny, int(round(p[2])) % nz))
    return pts


def run_grains(S, w, steps, nsamples, seed, flat=False, dtype="f32"):
    rng = np.random.default_rng(seed)
    print(f"full size {w.shape} grains={len(w.radii)} steps={steps}", flush=True)
    with S.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, dtype=dtype, coupling="local",
                kernel="tiled", zchunk=ZCHUNK, dt=w.dt) as s:
        assert s.info()["zchunk"] == ZCHUNK
        s.init_spheres(w.centers, w.radii)
        s.step(steps)
        got = s.get_field()
    pts = sample_points(rng, w.shape, w.centers, w.radii, nsamples, w.lam, flat)
    p = oracle.params((3, 3, 3), lam=w.lam, mu=w.mu, dt=w.dt, stencil=26, coupling="local",
                      eps=1e-300 if dtype == "f64" else 1e-30)
    field_at = lambda xyz: oracle.spheres_at(w.shape, w.centers, w.radii, xyz, lam=w.lam)
    ref = oracle.cone_step(p, w.shape, field_at, pts, steps)
    g = np.array([got[z, y, x] for x, y, z in pts], dtype=np.float64)
    interface = (ref > 1e-3) & (ref < 1 - 1e-3)
    assert interface.sum() > nsamples // 4
    return float(np.abs(g - ref).max())


def test_grain256_bench_configuration(S):
    from paper_1910_05180_amd import inputs
    err = run_grains(S, inputs.sphere256(mu=0.02), 6, 2000, 11)
    assert err <= 1e-5


def test_grains512_bench_configuration(S):
    from paper_1910_05180_amd import inputs
    err = run_grains(S, inputs.grains512(), 3, 1000, 12)
    assert err <= 1e-5


@pytest.mark.parametrize("dtype,nx,tol", [("f32", 32767, 1e-5), ("f64", 16383, 1e-12)])
def test_plane_at_the_32_bit_offset_limit(S, dtype, nx, tol):
    """The largest z-plane spfm_create accepts: nx x 16384 points, just under
    2^31 bytes, so in-plane byte offsets reach the top of their 32-bit range
    (3 planes; 1.6e9 FP32 or 8.1e8 FP64 points).  Grains sit at the corners
    of the plane and in its middle; sampled outputs after 2 steps against the
    oracle's dependency cones."""
    from types import SimpleNamespace
    w = SimpleNamespace(shape=(3, 16384, nx), lam=4.0, mu=0.02, dt=0.1,
                        centers=[(nx - 27.0, 16360.0, 1.0), (25.0, 16350.0, 0.0), (nx - 67.0, 30.0, 2.0),
                                 (nx / 2, 8000.0, 1.0)],
                        radii=[30.0, 24.0, 28.0, 40.0])
    err = run_grains(S, w, 2, 1000, 14, flat=True, dtype=dtype)
    assert err <= tol


def test_grain256_fp64_plain_one_step_everywhere(S):
    """The FP64 plain kernel of the metric, one step, every point of 256^3."""
    from paper_1910_05180_amd import inputs
    w = inputs.sphere256(mu=0.02)
    phi0 = oracle.init_spheres(w.shape, w.centers, w.radii, lam=w.lam)
    p = oracle.params(w.shape, lam=w.lam, mu=w.mu, dt=w.dt, stencil=26, coupling="local",
                      eps=1e-300)
    ref = oracle.step(p, phi0, 1)
    with S.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, dtype="f64", coupling="local",
                kernel="plain", dt=w.dt, eps=1e-300) as s:
        s.set_field(phi0)
        s.step(1)
        got = s.get_field()
    assert np.abs(got - ref).max() <= 1e-12


def test_grains512_reductions_full_field_and_crop(S):
    """The FP64 compensated reductions of the diagnostics on the 512^3 grains
    after a few steps: against a long-double sum of the whole field (its error
    bound, about log2(N) 2^-64 of the sum, is far below the bar) and, on a
    128^3 crop stepped as a grid of its own, against the oracle's exactly
    rounded sums."""
    from paper_1910_05180_amd import inputs
    w = inputs.grains512()
    print(f"reductions {w.shape} grains={len(w.radii)}", flush=True)
    with S.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, dtype="f32", coupling="local",
                kernel="tiled", zchunk=ZCHUNK, dt=w.dt) as s:
        s.init_spheres(w.centers, w.radii)
        s.step(4)
        d = s.diagnostics()
        f = s.get_field()
    v = f.astype(np.float64)
    ref_phi = float(np.sum(v.astype(np.longdouble)))
    ref_x = float(np.sum((v * (1.0 - v)).astype(np.longdouble)))
    del v
    assert abs(d["sum_phi"] - ref_phi) <= 1e-15 * ref_phi
    assert abs(d["sum_x"] - ref_x) <= 1e-15 * ref_x
    assert d["phase_volume"] == pytest.approx(ref_phi, rel=1e-15)
    assert d["interface_area"] == pytest.approx(4.0 / w.lam * ref_x, rel=1e-15)
    # a 128^3 crop holding grains and matrix, as a periodic grid of its own
    crop = np.ascontiguousarray(f[128:256, 192:320, 256:384])
    del f
    with S.Spfm(crop.shape, lam=w.lam, mu=w.mu, stencil=26, dtype="f32", coupling="local",
                kernel="tiled", dt=w.dt) as s:
        s.set_field(crop)
        s.step(3)
        dc = s.diagnostics()
        g = s.get_field().astype(np.float64)
    s1, s2 = oracle.exact_sums(g)
    assert 0.0 < s1 < g.size and s2 > 0.0
    assert abs(dc["sum_phi"] - s1) <= 1e-15 * s1
    assert abs(dc["sum_x"] - s2) <= 1e-15 * s2


def test_reductions_beyond_2_31_points(S):
    """The FP64 compensated reductions over 2.7e9 points (5 planes of the
    largest FP32 z-plane): the sum of phi agrees with an accurate host sum of
    the downloaded field, and min and max are exact."""
    import math
    shape = (5, 16384, 32767)
    with S.Spfm(shape, lam=4.0, mu=0.0, stencil=26, dtype="f32", kernel="tiled", dt=0.1) as s:
        s.init_spheres([(32740.0, 16360.0, 1.0), (16000.0, 8000.0, 1.0), (900.0, 300.0, 0.0)],
                       [300.0, 2500.0, 700.0])
        s.step(2)
        d = s.diagnostics()
        phi = s.get_field()
    # float32 values are exact in float64; numpy sums each 2^12-element chunk
    # pairwise (error below 12 ulps of the chunk's sum for these nonnegative
    # values) and fsum adds the chunk sums exactly rounded, so the reference is
    # within 1.4e-15 of the exact sum, relative
    flat = phi.reshape(-1)
    n = flat.size
    assert n > 2 ** 31
    parts = []
    for i in range(0, n, 1 << 26):
        ch = flat[i:i + (1 << 26)].astype(np.float64)
        m = ch.size - ch.size % 4096
        parts.extend(ch[:m].reshape(-1, 4096).sum(axis=1).tolist())
        parts.extend(ch[m:].tolist())
    exact = math.fsum(parts)
    print(f"reductions over {n} points: device {d['sum_phi']!r} exact {exact!r}", flush=True)
    assert d["sum_phi"] == pytest.approx(exact, rel=2e-15)
    assert d["phi_min"] == float(flat.min()) and d["phi_max"] == float(flat.max())
