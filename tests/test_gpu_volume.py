"""GPU parity of the constant-volume stepping (Sec. 3.3), the box particle and
the phi = 1/2 contour statistics against the oracle, and the cube relaxation
study of Fig. 9 on the device."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import as_f32_input, stable_dt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def sphere_field(R=10.0, n=32, lam=3.0):
    shape = (n, n, n)
    return oracle.init_spheres(shape, [(n / 2 + 0.3, n / 2 - 0.2, n / 2 + 0.1)], [R], lam=lam)


@pytest.mark.parametrize("kernel", ["plain", "tiled"])
@pytest.mark.parametrize("coupling,interp", [("local", "h3"), ("global", "h3"), ("cf", "h3"),
                                             ("cf", "h5")])
@pytest.mark.parametrize("dtype,steps,tol,mtol", [("f64", 60, 1e-12, 1e-11), ("f32", 200, 1e-5, 1e-4)])
def test_constant_volume_matches_oracle(S, kernel, coupling, interp, dtype, steps, tol, mtol):
    lam = 3.0
    phi0 = sphere_field(lam=lam)
    eps = 1e-300 if dtype == "f64" else 1e-30
    p = oracle.params(phi0.shape, lam=lam, stencil=26, coupling=coupling, u=(1.0, 2.0, 0.0),
                      eps=eps, interp=interp, mu=-0.2)
    p.dt = stable_dt(p)
    if dtype == "f32":
        phi0 = as_f32_input(phi0)
    print(f"case {coupling}+{interp} {kernel} {dtype} steps={steps}", flush=True)
    ref, mu = oracle.step_constant_volume(p, phi0, steps)
    with S.Spfm(phi0.shape, lam=lam, mu=-0.2, stencil=26, dtype=dtype, coupling=coupling,
                u=(1.0, 2.0, 0.0), eps=eps, C_Gamma=p.C_Gamma, kernel=kernel, dt=p.dt,
                interp=interp, conserve_volume=True) as s:
        s.set_field(phi0)
        assert math.isnan(s.diagnostics()["mu"])
        s.step(steps)
        d = s.diagnostics()
        got = s.get_field().astype(np.float64)
    assert float(np.abs(got - ref).max()) <= tol
    assert abs(d["mu"] / mu[-1] - 1.0) <= mtol


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_constant_volume_conserves_the_sum(S, dtype, tol):
    import torch
    phi0 = sphere_field()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        with S.Spfm(phi0.shape, lam=3.0, mu=-0.2, stencil=26, dtype=dtype, conserve_volume=True,
                    stream=st) as s:
            s.set_field(phi0)
            v0 = s.diagnostics()["sum_phi"]
            s.step(500)                     # graph replays of the step and its correction
            d = s.diagnostics()
    assert abs(d["sum_phi"] / v0 - 1.0) <= tol
    assert d["mu"] < 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("coupling,interp", [("local", "h3"), ("cf", "h5")])
def test_constant_volume_does_not_depend_on_the_schedule(S, dtype, coupling, interp):
    """The tiled step forms exact sums per work item: one-plane chunks on 96^3
    give more than 1024 items (added in a pass of their own before the
    correction, which follows every step), 64-plane chunks a few hundred (every
    step applies the previous one's correction as it reads), the size rule its
    own choice; the plain kernel's path sums 1024 block partials.  The fields
    after 40 steps and mu agree bit for bit among the tiled runs, and with the
    plain kernel's mu to the rounding of the step itself."""
    n, lam = 96, 3.0
    phi0 = oracle.init_spheres((n, n, n), [(47.3, 50.2, 45.1)], [20.0], lam=lam)
    if dtype == "f32":
        phi0 = as_f32_input(phi0)
    eps = 1e-300 if dtype == "f64" else 1e-30
    out = {}
    for name, kw in (("z1", dict(kernel="tiled", zchunk=1)), ("z64", dict(kernel="tiled", zchunk=64)),
                     ("auto", dict(kernel="auto")), ("plain", dict(kernel="plain"))):
        print(f"case cv schedule {dtype} {coupling}+{interp} {name}", flush=True)
        with S.Spfm(phi0.shape, lam=lam, mu=-0.2, stencil=26, dtype=dtype, coupling=coupling,
                    interp=interp, eps=eps, conserve_volume=True, **kw) as s:
            s.set_field(phi0)
            s.step(40)
            inf = s.info()
            out[name] = (s.get_field(), s.diagnostics()["mu"], inf["zchunk"], inf["tile_x"], inf["tile_y"])
    assert out["z1"][2] == 1 and out["z64"][2] == 64
    for name in ("z64", "auto"):
        assert np.array_equal(out[name][0], out["z1"][0]), name
        assert out[name][1] == out["z1"][1], name
        assert out[name][3:] == out["z1"][3:], name   # the untuned tile shape
    assert abs(out["plain"][1] / out["z1"][1] - 1.0) <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_constant_volume_equals_separate_correction(S, dtype):
    """One launch per step (the correction of each step applied by the next
    one as it reads, 4-plane chunks: 512 work items on 64^3) against a step and
    a correction launch per step (1-plane chunks: 2048 items): equal fields and
    mu bit for bit after 1, 2 and 3 steps, after 40 steps on a stream (graph
    replays of the fused launches), and across consecutive calls."""
    import torch
    n, lam = 64, 3.0
    phi0 = oracle.init_spheres((n, n, n), [(31.3, 30.2, 33.1), (10.0, 50.0, 12.0)], [15.0, 6.0], lam=lam)
    if dtype == "f32":
        phi0 = as_f32_input(phi0)
    eps = 1e-300 if dtype == "f64" else 1e-30
    for calls in ((1,), (2,), (3,), (40,), (3, 5, 34)):
        out = []
        for zc in (1, 4):
            print(f"case fused cv {dtype} calls={calls} zchunk={zc}", flush=True)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                with S.Spfm(phi0.shape, lam=lam, mu=-0.2, stencil=26, dtype=dtype, coupling="local",
                            eps=eps, conserve_volume=True, kernel="tiled", zchunk=zc, stream=st) as s:
                    s.set_field(phi0)
                    for m in calls:
                        s.step(m)
                    out.append((s.get_field(), s.diagnostics()))
        assert np.array_equal(out[0][0], out[1][0]), calls
        assert out[0][1]["mu"] == out[1][1]["mu"], calls
        assert out[0][1]["step"] == out[1][1]["step"] == sum(calls)
        assert out[0][1]["phase_volume"] == out[1][1]["phase_volume"]


def test_contour_stats_match_oracle(S):
    phi0 = sphere_field(R=12.0, n=40)
    p = oracle.params(phi0.shape, lam=3.0)
    eps, Rm, Rmin, Rmax, c, npts = oracle.sphericity(p, phi0)
    with S.Spfm(phi0.shape, lam=3.0, dtype="f64") as s:
        s.set_field(phi0)
        got = s.contour_stats()
    assert got["points"] == npts
    assert np.abs(np.array(got["centre"]) - c).max() < 1e-12
    for k, v in (("R_mean", Rm), ("R_min", Rmin), ("R_max", Rmax)):
        assert abs(got[k] - v) < 1e-12 * v, k
    assert abs(got["eps_eff"] - eps) < 1e-9


def test_init_box_matches_oracle(S):
    shape, lo, hi = (30, 34, 40), (8.3, 10.0, 7.6), (31.3, 24.0, 20.6)
    ref = oracle.init_box(shape, lo, hi, lam=3.0)
    for dtype, tol in (("f64", 1e-14), ("f32", 6e-8)):
        with S.Spfm(shape, lam=3.0, dtype=dtype) as s:
            s.init_box(lo, hi)
            assert float(np.abs(s.get_field().astype(np.float64) - ref).max()) <= tol


def relaxed_cube(S, *, lam, coupling, steps, n=60, edge=30.0, dtype="f32", u=(1.0, 0.0, 0.0), dt=None):
    """Fig. 9: a cube particle relaxed at constant volume; returns the contour
    statistics and the final driving force."""
    import torch
    lo = (n - edge) / 2 + 0.25
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        with S.Spfm((n, n, n), lam=lam, mu=-0.1, stencil=26, dtype=dtype, coupling=coupling, u=u, dt=dt,
                    conserve_volume=True, stream=st) as s:
            s.init_box((lo, lo, lo), (lo + edge, lo + edge, lo + edge))
            s.step(steps)
            d = s.diagnostics()
            c = s.contour_stats()
    return c, d


def test_cube_relaxes_to_a_sphere_at_lambda_4(S):
    """TI_n, lambda~ = 4: the relaxed particle is a sphere to the resolution of
    the contour measure (the paper reports below 3e-4 for every model), and its
    mu is the Gibbs-Thomson value of the volume-equivalent sphere."""
    c, d = relaxed_cube(S, lam=4.0, coupling="local", steps=3000)
    RV = oracle.sphere_radius_from_volume(d["phase_volume"], 4.0)
    print(f"cube lam=4 TI_n: eps={c['eps_eff']:.3e} R_mean={c['R_mean']:.3f} RV={RV:.3f} "
          f"mu={d['mu']:.5f} GT={-2 / RV:.5f}", flush=True)
    assert c["eps_eff"] < 5e-4
    assert abs(d["mu"] / (-2.0 / RV) - 1.0) < 2e-2


def test_cf_cube_stays_anisotropic_where_ti_relaxes(S):
    """Fig. 9b: at lambda~ = 2 the CF particle keeps partly pinned faces, its
    anisotropy far above that of TI_n."""
    c_ti, _ = relaxed_cube(S, lam=2.0, coupling="local", steps=3000)
    c_cf, _ = relaxed_cube(S, lam=2.0, coupling="cf", steps=3000)
    print(f"cube lam=2: TI_n eps={c_ti['eps_eff']:.3e}, CF eps={c_cf['eps_eff']:.3e}", flush=True)
    assert c_ti["eps_eff"] < 1e-3
    assert c_cf["eps_eff"] > 10 * c_ti["eps_eff"]


FIG9B_MODELS = {"TI_n": ("local", (1.0, 0.0, 0.0)), "TI_100": ("global", (1.0, 0.0, 0.0)),
                "TI_110": ("global", (1.0, 1.0, 0.0)), "TI_120": ("global", (1.0, 2.0, 0.0)),
                "CF": ("cf", (1.0, 0.0, 0.0))}


def fig9b_eps(S, lam, model, T=300.0):
    """eps_eff of the cube relaxed for T time units, dt half the explicit bound
    (at most 0.1)."""
    coupling, u = FIG9B_MODELS[model]
    dt = min(0.1, 0.5 * S.stable_dt(26, coupling, u, None, lam, 1.0, 1.0, 0.2, 1.0))
    steps = int(math.ceil(T / dt))
    print(f"case fig9b lam={lam} {model} dt={dt:.3g} steps={steps}", flush=True)
    c, _ = relaxed_cube(S, lam=lam, coupling=coupling, u=u, dt=dt, steps=steps)
    print(f"eps_eff {c['eps_eff']:.3e}", flush=True)
    return c["eps_eff"]


def test_fig9b_every_model_is_nearly_isotropic_at_lambda_4(S):
    """Sec. 3.3: at lambda~ = 4 every model relaxes the cube to a sphere with a
    sphericity error below 3e-4 (measured 2.1e-4 to 2.6e-4)."""
    for model in FIG9B_MODELS:
        assert fig9b_eps(S, 4.0, model) < 3e-4, model


def test_fig9b_ti_hkl_pins_below_1_3_unless_aligned_with_the_faces(S):
    """Sec. 3.3: below lambda~ = 1.3 the TI_<hkl> models whose directions of
    restored invariance miss the cube's faces keep it partly pinned (TI_<110>
    7%, TI_<120> 5% at lambda~ = 1.2), while TI_<100>, aligned with the faces,
    and TI_n relax it (below 1%); CF stays a pinned cube (24%)."""
    e = {m: fig9b_eps(S, 1.2, m) for m in FIG9B_MODELS}
    assert e["TI_110"] > 3e-2 and e["TI_120"] > 3e-2
    assert e["TI_100"] < 1e-2 and e["TI_n"] < 1e-2
    assert e["CF"] > 0.1


def test_fig9b_ti_n_anisotropy_grows_gradually(S):
    """Sec. 3.3: the TI_n sphericity error is low and grows gradually as the
    profile sharpens (measured 2.1e-4, 5.8e-4, 2.0e-3, 5.0e-3, 9.2e-3 at
    lambda~ = 4, 2, 1.5, 1.2, 1)."""
    e = [fig9b_eps(S, lam, "TI_n") for lam in (4.0, 2.0, 1.5, 1.2, 1.0)]
    assert all(b > a for a, b in zip(e, e[1:]))
    assert e[-1] < 1.5e-2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ray_radii_match_the_oracle(S, dtype):
    """Radii along 500 seeded rays from the barycentre of a grain built by the
    oracle, on the device and in the oracle from the same (for FP32, the same
    FP32-rounded) field: the same march and bisection, so within 1e-9."""
    shape, R, cen = (48, 44, 52), 13.0, (25.3, 21.6, 23.9)
    phi = oracle.init_spheres(shape, [cen], [R], lam=3.0)
    if dtype == "f32":
        phi = phi.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(17)
    d = rng.normal(size=(500, 3))
    with S.Spfm(shape, lam=3.0, stencil=26, dtype=dtype) as s:
        s.set_field(phi)
        got = s.ray_radii(d, centre=cen)
        dflt = s.ray_radii(d[:10])     # centre: the contour barycentre
        same = s.ray_radii(d[:10], centre=s.contour_stats()["centre"])
    ref = oracle.ray_radii(phi, cen, d)
    assert not np.isnan(ref).any()
    assert float(np.abs(got - ref).max()) <= 1e-9
    assert np.array_equal(dflt, same)


def test_ray_radii_exact_for_a_linear_psi_on_the_device(S):
    shape = (40, 40, 40)
    n = np.array([1.0, 0.4, -0.3])
    n /= np.linalg.norm(n)
    centre = np.array([20.3, 19.7, 20.1])
    c0 = float(n @ centre) + 9.3
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 1.0 / (1.0 + np.exp(n[0] * xx + n[1] * yy + n[2] * zz - c0))
    rng = np.random.default_rng(5)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d = d[d @ n >= 0.55][:100]
    with S.Spfm(shape, lam=4.0, stencil=26, dtype="f64") as s:
        s.set_field(phi)
        got = s.ray_radii(d, centre=centre)
        outside = s.ray_radii(-d[:3], centre=centre + 12.0 * n)
    assert float(np.abs(got - (c0 - n @ centre) / (d @ n)).max()) < 1e-9
    assert np.isnan(outside).all()


def test_ray_radii_reject_bad_arguments(S):
    with S.Spfm((16, 16, 16), lam=3.0, stencil=26, dtype="f32") as s:
        with pytest.raises(S.SpfmError):
            s.ray_radii(np.array([[0.0, 0.0, 0.0]]), centre=(8.0, 8.0, 8.0))
        with pytest.raises(S.SpfmError):
            s.ray_radii(np.array([[1.0, 0.0, 0.0]]), centre=(8.0, float("nan"), 8.0))
    with S.Spfm((16, 16, 16), lam=3.0, stencil=26, dtype="f32", walls=1,
                wall_sin=(0, 0, 0, 0, 0, 0)) as s:
        with pytest.raises(S.SpfmError):
            s.ray_radii(np.array([[1.0, 0.0, 0.0]]), centre=(8.0, 8.0, 8.0))
