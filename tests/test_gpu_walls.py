"""GPU parity of the contact-angle walls (Sec. 2.2, Eq. 7) against the oracle,
and the kinetics of the paper's orientation study (Sec. 3.2) on the device.

The oracle fills the ghost layers wall after wall (Eq. 7 as printed); the
library applies the composed shift of a ghost's walls at once.  The two agree
to rounding, so the bars are those of the periodic parity tests: FP64 within
1e-12, FP32 within 1e-5 of the FP64 oracle from the same FP32-rounded field."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import as_f32_input, sphere12, stable_dt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def rot001(theta):
    return (math.cos(theta), math.sin(theta), 0.0)


def rot011(theta):
    return (math.cos(theta), math.sin(theta) / math.sqrt(2.0), math.sin(theta) / math.sqrt(2.0))


def run_pair(S, phi0, steps, *, walls, sa, dtype, kernel, stencil=26, coupling="local", lam=2.5,
             mu=0.02, u=(1.0, 2.0, 0.0)):
    eps = 1e-300 if dtype == "f64" else 1e-30
    shape = phi0.shape
    p = oracle.params(shape, lam=lam, mu=mu, stencil=stencil, coupling=coupling, u=u, eps=eps)
    p.dt = stable_dt(p)
    if dtype == "f32":
        phi0 = as_f32_input(phi0)
    print(f"case walls={walls} shape={shape} steps={steps} {dtype} {kernel} S={stencil} {coupling}",
          flush=True)
    ref = oracle.step_walls(p, phi0, walls, sa, steps)
    with S.Spfm(shape, lam=lam, mu=mu, stencil=stencil, dtype=dtype, coupling=coupling, u=u,
                eps=eps, C_Gamma=p.C_Gamma, kernel=kernel, dt=p.dt, walls=walls, wall_sin=sa) as s:
        s.set_field(phi0)
        s.step(steps)
        got = s.get_field().astype(np.float64)
    return float(np.abs(got - ref).max())


FRONT_SHAPE = (9, 11, 37)
FRONT_N = rot011(0.5)


def front_field(lam=2.5):
    return oracle.front(FRONT_SHAPE, FRONT_N, 1.3, lam=lam)


@pytest.mark.parametrize("kernel", ["plain", "tiled"])
@pytest.mark.parametrize("stencil", [6, 18, 26])
@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
def test_walled_front_fp64(S, kernel, stencil, coupling):
    err = run_pair(S, front_field(), 30, walls=7, sa=oracle.front_sin_alpha(FRONT_N), dtype="f64",
                   kernel=kernel, stencil=stencil, coupling=coupling)
    assert err <= 1e-12


@pytest.mark.parametrize("kernel", ["plain", "tiled"])
@pytest.mark.parametrize("stencil", [6, 18, 26])
@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
def test_walled_front_fp32(S, kernel, stencil, coupling):
    err = run_pair(S, front_field(), 150, walls=7, sa=oracle.front_sin_alpha(FRONT_N), dtype="f32",
                   kernel=kernel, stencil=stencil, coupling=coupling)
    assert err <= 1e-5


@pytest.mark.parametrize("walls,sa", [
    (4, (0.0, 0.0, 0.0, 0.0, -0.3, 0.45)),       # z walled, x and y periodic
    (3, (0.2, -0.1, 0.5, 0.0, 0.0, 0.0)),         # x and y walled
    (1, (-0.6, 0.6, 0.0, 0.0, 0.0, 0.0)),         # x walled only
])
@pytest.mark.parametrize("dtype,steps,tol", [("f64", 20, 1e-12), ("f32", 100, 1e-5)])
def test_walls_on_some_axes_with_a_grain(S, walls, sa, dtype, steps, tol):
    """A grain reaching towards walls whose angles it does not match."""
    for kernel in ("plain", "tiled"):
        err = run_pair(S, sphere12(), steps, walls=walls, sa=sa, dtype=dtype, kernel=kernel, lam=2.0)
        assert err <= tol, (kernel, err)


@pytest.mark.parametrize("shape,walls", [((3, 3, 3), 7), ((3, 5, 4), 1), ((4, 3, 70), 6),
                                         ((33, 4, 5), 5)])
def test_walls_on_small_grids(S, shape, walls):
    n = (0.8, -0.5, 0.3)
    phi0 = oracle.front(shape, n, 0.2, lam=3.0) if walls == 7 else \
        np.clip(oracle.front(shape, (1.0, 0.0, 0.0), 0.0, lam=3.0) * 0.9 + 0.05, 0, 1)
    sa = oracle.front_sin_alpha(n)
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
        for kernel in ("plain", "tiled"):
            err = run_pair(S, phi0, 10, walls=walls, sa=sa, dtype=dtype, kernel=kernel, lam=3.0)
            assert err <= tol, (dtype, kernel, err)


@pytest.mark.parametrize("shape,walls,n", [((65533, 3, 3), 4, (0.0, 0.0, 1.0)),
                                           ((3, 262138, 3), 2, (0.0, 1.0, 0.0))])
def test_walled_axes_at_their_maximum_length(S, shape, walls, n):
    """A walled axis whose two ghost layers make the stored length the
    largest accepted (nz = 65535, ny = 262140); the front varies along it."""
    phi0 = np.clip(oracle.front(shape, n, 0.0, lam=3.0) * 0.9 + 0.05, 0, 1)
    sa = oracle.front_sin_alpha((0.8, -0.5, 0.3))
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
        for kernel in ("plain", "tiled"):
            err = run_pair(S, phi0, 5, walls=walls, sa=sa, dtype=dtype, kernel=kernel, lam=3.0)
            assert err <= tol, (dtype, kernel, err)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_walled_front_stays_put_for_ti_along_its_normal(S, dtype, tol):
    """TI with u = n at mu = 0 keeps the ideal tilted front (Sec. 2.2), walls included."""
    n = rot011(0.6)
    phi0 = oracle.front(FRONT_SHAPE, n, 0.7, lam=3.0)
    with S.Spfm(FRONT_SHAPE, lam=3.0, mu=0.0, stencil=26, dtype=dtype, coupling="global", u=n,
                walls=7, wall_sin=oracle.front_sin_alpha(n)) as s:
        s.set_field(phi0)
        start = s.get_field().astype(np.float64)
        s.step(100)
        got = s.get_field().astype(np.float64)
    assert float(np.abs(got - start).max()) <= tol


def test_set_get_and_diagnostics_use_the_interior(S):
    phi0 = front_field()
    with S.Spfm(FRONT_SHAPE, lam=2.5, dtype="f64", walls=5,
                wall_sin=oracle.front_sin_alpha(FRONT_N)) as s:
        s.set_field(phi0)
        assert np.array_equal(s.get_field(), phi0)
        d = s.diagnostics()
        assert d["sum_phi"] == pytest.approx(math.fsum(phi0.ravel()), rel=1e-15, abs=1e-12)
        assert s.info()["walls"] == 5
        s.step(3)
        d = s.diagnostics()
        assert d["sum_phi"] == pytest.approx(math.fsum(s.get_field().ravel()), rel=1e-15, abs=1e-12)


def test_init_front_matches_the_oracle(S):
    n = (0.9, -0.2, 0.35)
    for dtype, tol in (("f64", 1e-14), ("f32", 6e-8)):
        with S.Spfm(FRONT_SHAPE, lam=2.5, dtype=dtype, walls=7,
                    wall_sin=oracle.front_sin_alpha(n)) as s:
            s.init_front(n, -0.4)
            got = s.get_field().astype(np.float64)
        assert float(np.abs(got - oracle.front(FRONT_SHAPE, n, -0.4, lam=2.5)).max()) <= tol


def test_init_front_needs_walls_where_the_front_varies(S):
    with S.Spfm((8, 8, 8), lam=2.5, walls=1, wall_sin=(-1, 1, 0, 0, 0, 0)) as s:
        s.init_front((1.0, 0.0, 0.0))
        with pytest.raises(S.SpfmError):
            s.init_front((1.0, 0.5, 0.0))


def front_velocity(S, n, *, dtype, mu0=0.05, lam=4.0, shape=(10, 10, 120), dt=0.05, warm=400,
                   steps=1600):
    """x-velocity of a walled planar front driven by mu = mu0 n_x (Sec. 3.2)."""
    import torch
    nv = np.asarray(n) / np.linalg.norm(n)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        with S.Spfm(shape, lam=lam, mu=mu0 * nv[0], stencil=26, dtype=dtype, coupling="local",
                    dt=dt, walls=7, wall_sin=oracle.front_sin_alpha(nv), stream=st) as s:
            s.init_front(nv, 20.0)
            s.step(warm)
            d0 = s.diagnostics()
            s.step(steps)
            d1 = s.diagnostics()
    vn = (d1["interface_position"] - d0["interface_position"]) / (d1["time"] - d0["time"])
    return vn / nv[0]


@pytest.mark.parametrize("axis,deg", [("001", 0), ("001", 15), ("001", 30), ("001", 45),
                                      ("011", 15), ("011", 30), ("011", 45)])
def test_orientation_study_velocity(S, axis, deg):
    """120 x 10 x 10 box, TI_n, lambda = 4: every orientation moves its front
    along x at -M mu0 / Gamma (the paper reports errors below 0.1 % at this
    resolution; the forward-Euler step here adds its own)."""
    th = math.radians(deg)
    n = rot001(th) if axis == "001" else rot011(th)
    vx = front_velocity(S, n, dtype="f32")
    print(f"theta[{axis}]={deg} vx={vx:.6f} err={vx / -0.05 - 1:+.2e}", flush=True)
    assert abs(vx / -0.05 - 1.0) < 2e-3


def test_orientation_study_fp32_equals_fp64(S):
    n = rot011(math.radians(35))
    v32 = front_velocity(S, n, dtype="f32", steps=800)
    v64 = front_velocity(S, n, dtype="f64", steps=800)
    assert abs(v32 / v64 - 1.0) < 1e-4


ORIENTATIONS = [rot001(math.radians(d)) for d in (0, 15, 30, 45)] + \
               [rot011(math.radians(d)) for d in (15, 30, 45)]


def test_walled_batch_equals_single_contexts(S):
    """The orientation study as one batch (seven 120 x 10 x 10 walled grids,
    each with its own wall angles and driving force) equals seven separate
    walled contexts bit for bit, field and front position."""
    shape, lam, mu0, dt, steps = (10, 10, 120), 4.0, 0.05, 0.05, 300
    ns = [np.asarray(n) / np.linalg.norm(n) for n in ORIENTATIONS]
    sins = [oracle.front_sin_alpha(n) for n in ns]
    mus = [mu0 * n[0] for n in ns]
    print(f"case walled batch of {len(ns)} orientations, {steps} steps", flush=True)
    with S.SpfmBatch([shape] * len(ns), lam=lam, mu=mus, stencil=26, coupling="local", dt=dt,
                     walls=7, wall_sin=sins) as b:
        b.init_front(ns, [20.0] * len(ns))
        b.step(steps)
        db = b.diagnostics()
        fields = [b.get_field(i) for i in range(len(ns))]
    for i, n in enumerate(ns):
        with S.Spfm(shape, lam=lam, mu=mus[i], stencil=26, dtype="f32", coupling="local", dt=dt,
                    walls=7, wall_sin=sins[i], kernel="tiled") as s:
            s.init_front(n, 20.0)
            s.step(steps)
            d = s.diagnostics()
            assert np.array_equal(s.get_field(), fields[i]), i
        assert d["interface_position"] == db[i]["interface_position"], i
        assert d["sum_phi"] == db[i]["sum_phi"], i


@pytest.mark.parametrize("walls", [1, 6, 7])
def test_walled_batch_of_uneven_grids_matches_the_oracle(S, walls):
    """Grids of different, ragged sizes with the same walled axes, each with its
    own wall angles, against the oracle's wall-after-wall fill (FP32 bar)."""
    shapes = [(9, 11, 37), (5, 6, 20), (12, 3, 70)] if walls != 1 else [(9, 11, 37), (5, 6, 20)]
    lam, mu = 2.5, 0.02
    rng = np.random.default_rng(7)
    sas, fields, ps = [], [], []
    for shape in shapes:
        n = rng.normal(size=3)
        n[[d for d in range(3) if not (walls >> d) & 1]] = 0.0
        n[0] = abs(n[0]) + 0.5 if walls & 1 else n[0]
        n = n / np.linalg.norm(n)
        sa = oracle.front_sin_alpha(n)
        sas.append(sa)
        fields.append(as_f32_input(oracle.front(shape, n, 0.7, lam=lam)))
        p = oracle.params(shape, lam=lam, mu=mu, stencil=26, coupling="local", eps=1e-30)
        ps.append(p)
    dt = min(stable_dt(p) for p in ps)
    steps = 60
    print(f"case walled batch walls={walls} shapes={shapes}", flush=True)
    with S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling="local", dt=dt, walls=walls,
                     wall_sin=sas) as b:
        for i, f in enumerate(fields):
            b.set_field(i, f)
            assert np.array_equal(b.get_field(i), f.astype(np.float32))
        b.step(steps)
        got = [b.get_field(i).astype(np.float64) for i in range(len(shapes))]
    for i, p in enumerate(ps):
        p.dt = dt
        ref = oracle.step_walls(p, fields[i], walls, sas[i], steps)
        assert float(np.abs(got[i] - ref).max()) <= 1e-5, i


@pytest.mark.parametrize("coupling", ["local", "cf"])
def test_walled_batch_results_do_not_depend_on_the_zchunk(S, coupling):
    """The kernel computes the wall ghosts as it stages each plane, whatever
    z-chunk a block starts at: a small walled batch (chunks of 4 planes by the
    size rule) and the same batch with 32-plane and 7-plane chunks give bitwise
    the same fields."""
    shapes = [(9, 11, 37), (5, 6, 20), (12, 3, 70)]
    lam, mu = 2.5, 0.02
    rng = np.random.default_rng(11)
    sas, fields = [], []
    for shape in shapes:
        n = rng.normal(size=3)
        n[0] = abs(n[0]) + 0.5
        n = n / np.linalg.norm(n)
        sas.append(oracle.front_sin_alpha(n))
        fields.append(as_f32_input(oracle.front(shape, n, 0.7, lam=lam)))
    p = oracle.params(shapes[0], lam=lam, mu=mu, stencil=26, coupling=coupling, eps=1e-30)
    dt = stable_dt(p)
    out = {}
    for zc in (0, 32, 7):
        print(f"case walled batch {coupling} zchunk={zc}", flush=True)
        with S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling=coupling, dt=dt, walls=7,
                         wall_sin=sas, zchunk=zc) as b:
            for i, f in enumerate(fields):
                b.set_field(i, f)
            b.step(40)
            out[zc] = [b.get_field(i) for i in range(len(shapes))]
    for zc in (32, 7):
        for i in range(len(shapes)):
            assert np.array_equal(out[zc][i], out[0][i]), (zc, i)


# --- Fig. 8 at the paper's other two resolutions --------------------------------

def fig8_errors(S, lam, coupling, u=(1.0, 0.0, 0.0), warm_cells=0.5, window_cells=1.0, mu0=0.1):
    """Relative x-velocity errors of the seven orientations of Fig. 8 as one
    walled FP32 batch (120 x 10 x 10, 26 neighbours, mu = mu0 cos(theta), dt
    half the explicit bound), the front located by its psi = 0 crossings
    (bench.front_x, exact for the ideal profile at any lambda/dx)."""
    import bench
    bound = min(S.stable_dt(26, coupling, u, None, lam, 1.0, 1.0, mu0 * n[0], 1.0) for n in ORIENTATIONS)
    dt = min(0.05, 0.5 * bound)
    warm = int(math.ceil(warm_cells / mu0 / dt))
    steps = int(math.ceil(window_cells / mu0 / dt))
    print(f"case fig8 lam={lam} {coupling} u={u} dt={dt:.3g} steps={warm}+{steps}", flush=True)
    with S.SpfmBatch([(10, 10, 120)] * len(ORIENTATIONS), lam=lam, mu=[mu0 * n[0] for n in ORIENTATIONS],
                     stencil=26, coupling=coupling, u=u, dt=dt, walls=7,
                     wall_sin=[S.front_wall_sin(n) for n in ORIENTATIONS]) as b:
        b.init_front(ORIENTATIONS, [20.0] * len(ORIENTATIONS))
        b.step(warm)
        x0 = [bench.front_x(b.get_field(i)) for i in range(len(ORIENTATIONS))]
        b.step(steps)
        x1 = [bench.front_x(b.get_field(i)) for i in range(len(ORIENTATIONS))]
    errs = [(c - a) / (steps * dt) / (-mu0) - 1.0 for a, c in zip(x0, x1)]
    print(" ".join(f"{e:+.2e}" for e in errs), flush=True)
    return errs


def test_fig8_ti_n_is_frictionless_at_lambda_1(S):
    """Sec. 3.2: TI_n moves every orientation at -M mu0 / Gamma also at
    lambda = dx; what remains is the forward-Euler error (about 7e-5 at half
    the stability bound, the same in FP64)."""
    errs = fig8_errors(S, 1.0, "local")
    assert max(abs(e) for e in errs) < 2e-4


def test_fig8_continuum_field_pins_at_lambda_1(S):
    """Sec. 3.2: below lambda = 4 the CF model is pinned by the grid at every
    orientation (mu0 dx / Gamma = 0.1)."""
    errs = fig8_errors(S, 1.0, "cf")
    assert max(errs) < -0.999


def test_fig8_ti_hkl_is_exact_only_along_its_directions(S):
    """Sec. 3.2: a TI_<hkl> model moves fronts normal to its <hkl> directions
    at the expected velocity; misoriented ones not, and TI_<110> is pinned
    near [100] at lambda = dx.  (For TI_<100> the misoriented fronts here run
    5-21% fast over five cells, where the paper's text says slow.)"""
    e100 = fig8_errors(S, 1.0, "global", u=(1.0, 0.0, 0.0))
    assert abs(e100[0]) < 2e-4                      # [100]
    assert min(abs(e) for e in e100[1:]) > 0.02     # every other orientation
    e110 = fig8_errors(S, 1.0, "global", u=(1.0, 1.0, 0.0))
    assert abs(e110[3]) < 2e-4                      # 45 degrees about [001]: [110]
    assert e110[0] < -0.99                          # pinned along [100]


@pytest.mark.parametrize("deg", [0, 15])
def test_fig8_ti_n_at_lambda_half(S, deg):
    """Sec. 3.2: TI_n stays frictionless at lambda = dx / 2, the error that of
    the time step (dt = 1e-5, the paper's), in FP64.  FP32 storage resolves
    1 - phi only to 6e-8, and two cells behind this front the ideal profile's
    1 - phi is 1.1e-7: psi' and hence the local normal lose their accuracy
    there, and the FP32 front errs by up to about 2% (a bound of 5% guards that
    documented limit)."""
    import bench
    th = math.radians(deg)
    n = rot001(th)
    lam, mu0 = 0.5, 0.1
    dt = 0.5 * S.stable_dt(26, "local", n, None, lam, 1.0, 1.0, mu0 * n[0], 1.0)
    warm, steps = int(math.ceil(0.05 / mu0 / dt)), int(math.ceil(0.25 / mu0 / dt))
    errs = {}
    for dtype in ("f64", "f32"):
        print(f"case fig8 lam=0.5 TI_n {dtype} theta={deg} dt={dt:.3g} steps={warm}+{steps}", flush=True)
        with S.Spfm((10, 10, 120), lam=lam, mu=mu0 * n[0], stencil=26, dtype=dtype, coupling="local", dt=dt,
                    walls=7, wall_sin=S.front_wall_sin(n)) as s:
            s.init_front(n, 20.0)
            s.step(warm)
            x0 = bench.front_x(s.get_field())
            s.step(steps)
            x1 = bench.front_x(s.get_field())
        errs[dtype] = (x1 - x0) / (steps * dt) / (-mu0) - 1.0
        print(f"{dtype} err {errs[dtype]:+.3e}", flush=True)
    assert abs(errs["f64"]) < 1e-4
    assert abs(errs["f32"]) < 5e-2
