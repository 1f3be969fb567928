"""The resident step (one workgroup per grid holds the grid in LDS and takes
many steps per launch): equal bit for bit to the tiled step on the same grids,
and held to the oracle.

Batches whose grids all fit choose it by default, so the walled orientation
batch and the model-comparison slabs of the other tests run it too; here it is
compared with the tiled batched kernel explicitly, across couplings, stencils,
driving-force interpolations, walls, grid shapes that wrap onto themselves,
odd and even step counts (the output goes to the other buffer or back into the
same one) and runs longer than one launch's share of steps.  Grids cut into x
segments (one workgroup each, redundant halos, at most a halo's worth of steps
per launch) must give the same bits again."""
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


def rot011(theta):
    return (math.cos(theta), math.sin(theta) / math.sqrt(2.0), math.sin(theta) / math.sqrt(2.0))


def batch_fields(S, shapes, kernel, steps, init, **kw):
    with S.SpfmBatch(shapes, kernel=kernel, **kw) as b:
        assert b.kernel == kernel
        init(b)
        out = []
        for n in steps:
            b.step(n)
            out.append([b.get_field(i) for i in range(len(shapes))])
        d = b.diagnostics()
    return out, d


def assert_bitwise(a, b):
    for fa, fb in zip(a, b):
        for x, y in zip(fa, fb):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_orientation_batch_equals_tiled(S):
    """The seven walled 120 x 10 x 10 fronts of the orientation study (TI_n, 26
    neighbours), 1, 2, 97 and 300 more steps."""
    ns = [np.asarray(n) / np.linalg.norm(n) for n in
          [(1, 0, 0), rot011(math.radians(15)), rot011(math.radians(45)), (0.8, 0.6, 0.0)]]
    sins = [oracle.front_sin_alpha(n) for n in ns]
    kw = dict(lam=4.0, mu=[0.05 * n[0] for n in ns], stencil=26, coupling="local", dt=0.05, walls=7,
              wall_sin=sins)
    init = lambda b: b.init_front(ns, [20.0] * len(ns))
    print("case resident orientation batch", flush=True)
    r, dr = batch_fields(S, [(10, 10, 120)] * len(ns), "resident", [1, 2, 97, 300], init, **kw)
    t, dt_ = batch_fields(S, [(10, 10, 120)] * len(ns), "tiled", [1, 2, 97, 300], init, **kw)
    assert_bitwise(r, t)
    for a, b in zip(dr, dt_):
        assert a["interface_position"] == b["interface_position"] and a["step"] == 400


@pytest.mark.parametrize("coupling,interp", [("local", "h3"), ("global", "h3"), ("cf", "h3"),
                                             ("cf", "h5"), ("cf", "habel")])
@pytest.mark.parametrize("stencil", [6, 18, 26])
def test_slabs_equal_tiled(S, coupling, interp, stencil):
    """Periodic slabs of the model comparison and ragged small grids (including
    3^3, whose halo wraps onto itself) for every kernel variant."""
    shapes = [(3, 3, 64), (3, 3, 3), (5, 4, 3), (7, 11, 9), (12, 3, 33)]
    hkl = [(1, 0, 0), (1, 1, 1), (1, 0, 1), (2, 1, 1), (1, 2, 3)]
    lam = 2.5
    mu = 0.3 if coupling == "cf" else 0.04
    kw = dict(lam=lam, mu=mu, stencil=stencil, coupling=coupling, interp=interp, u=(1.0, 2.0, 0.0),
              dt=0.02)
    init = lambda b: b.init_planar(hkl, [0.3, 0.1, 0.7, 0.2, 0.5])
    print(f"case resident slabs {coupling}+{interp} S={stencil}", flush=True)
    r, _ = batch_fields(S, shapes, "resident", [7, 10], init, **kw)
    t, _ = batch_fields(S, shapes, "tiled", [7, 10], init, **kw)
    assert_bitwise(r, t)


def test_long_run_across_launches_equals_tiled(S):
    """More steps than one resident launch takes (4096): 4099 steps, then 5."""
    shapes = [(3, 3, 256)] * 3
    kw = dict(lam=[4.0, 3.0, 2.5], mu=[0.005, 0.01, 0.02], stencil=6, coupling="local", dt=0.05)
    init = lambda b: b.init_planar([(1, 0, 0)] * 3, [0.37] * 3)
    print("case resident 4099 + 5 steps", flush=True)
    r, dr = batch_fields(S, shapes, "resident", [4099, 5], init, **kw)
    t, dt_ = batch_fields(S, shapes, "tiled", [4099, 5], init, **kw)
    assert_bitwise(r, t)
    assert [d["interface_position"] for d in dr] == [d["interface_position"] for d in dt_]


@pytest.mark.parametrize("walls", [0, 1, 6, 7])
def test_batch_matches_oracle(S, walls):
    """Uneven grids with their own fronts or slabs against the oracle (FP32 bar)."""
    shapes = [(9, 11, 37), (5, 6, 20), (12, 3, 70)]
    lam, mu, steps = 2.5, 0.02, 60
    rng = np.random.default_rng(11 + walls)
    fields, sas, ps = [], [], []
    for shape in shapes:
        if walls:
            n = rng.normal(size=3)
            n[[d for d in range(3) if not (walls >> d) & 1]] = 0.0
            n[0] = abs(n[0]) + 0.5 if walls & 1 else n[0]
            n = n / np.linalg.norm(n)
            sas.append(oracle.front_sin_alpha(n))
            fields.append(as_f32_input(oracle.front(shape, n, 0.7, lam=lam)))
        else:
            fields.append(as_f32_input(oracle.init_spheres(shape, [(shape[2] / 2, shape[1] / 2, shape[0] / 2)],
                                                           [min(shape) / 2.5], lam=lam)))
        ps.append(oracle.params(shape, lam=lam, mu=mu, stencil=26, coupling="local", eps=1e-30))
    dt = min(stable_dt(p) for p in ps)
    print(f"case resident vs oracle walls={walls}", flush=True)
    kw = dict(walls=walls, wall_sin=sas) if walls else {}
    with S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling="local", dt=dt, kernel="resident",
                     **kw) as b:
        for i, f in enumerate(fields):
            b.set_field(i, f)
        b.step(steps)
        got = [b.get_field(i).astype(np.float64) for i in range(len(shapes))]
    for i, p in enumerate(ps):
        p.dt = dt
        ref = (oracle.step_walls(p, fields[i], walls, sas[i], steps) if walls
               else oracle.step(p, fields[i], steps))
        assert float(np.abs(got[i] - ref).max()) <= 1e-5, i


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
@pytest.mark.parametrize("walls", [0, 7])
def test_context_matches_oracle_and_tiled(S, dtype, tol, walls):
    """A single context with the resident kernel: within the bar of the oracle,
    and equal to the tiled kernel bit for bit (FP32 and FP64); set_mu between
    runs re-uploads its coefficients."""
    shape, lam = (10, 12, 40), 2.5
    eps = 1e-300 if dtype == "f64" else 1e-30
    n = np.asarray(rot011(0.4))
    sa = oracle.front_sin_alpha(n) if walls else None
    phi0 = (oracle.front(shape, n, 0.4, lam=lam) if walls else
            oracle.init_spheres(shape, [(20.3, 6.2, 5.1)], [4.5], lam=lam))
    start = phi0 if dtype == "f64" else as_f32_input(phi0)
    p = oracle.params(shape, lam=lam, mu=0.03, stencil=26, coupling="local", eps=eps)
    p.dt = stable_dt(p)
    ref = oracle.step_walls(p, start, walls, sa, 25) if walls else oracle.step(p, start, 25)
    p.mu = -0.02
    ref = oracle.step_walls(p, ref, walls, sa, 30) if walls else oracle.step(p, ref, 30)
    out = {}
    for kernel in ("resident", "tiled"):
        print(f"case resident context {dtype} walls={walls} {kernel}", flush=True)
        kw = dict(walls=walls, wall_sin=sa) if walls else {}
        with S.Spfm(shape, lam=lam, mu=0.03, stencil=26, dtype=dtype, coupling="local", eps=eps,
                    C_Gamma=p.C_Gamma, dt=p.dt, kernel=kernel, **kw) as s:
            assert s.info()["kernel"] == S.KERNEL_RESIDENT or kernel == "tiled"
            s.set_field(phi0)
            s.step(25)
            s.set_mu(-0.02)
            s.step(30)
            out[kernel] = s.get_field()
    assert float(np.abs(out["resident"].astype(np.float64) - ref).max()) <= tol
    assert np.array_equal(out["resident"], out["tiled"])


def segment_batch(S, shapes, segment, steps, init, kernel="resident", **kw):
    with S.SpfmBatch(shapes, kernel=kernel, segment=segment, **kw) as b:
        init(b)
        out = []
        for n in steps:
            b.step(n)
            out.append([b.get_field(i) for i in range(len(shapes))])
        info = b.info()
        d = b.diagnostics()
    return out, info, d


@pytest.mark.parametrize("segment", [(8, 4), (16, 8), (4, 32), (1, 1), (30, 3)])
def test_walled_orientation_segments_equal_tiled(S, segment):
    """The walled orientation batch (TI_n, 26 neighbours) cut into x segments:
    1, 2, 97 and 300 more steps equal the tiled kernel bit for bit."""
    ns = [np.asarray(n) / np.linalg.norm(n) for n in
          [(1, 0, 0), rot011(math.radians(15)), rot011(math.radians(45)), (0.8, 0.6, 0.0)]]
    sins = [oracle.front_sin_alpha(n) for n in ns]
    kw = dict(lam=4.0, mu=[0.05 * n[0] for n in ns], stencil=26, coupling="local", dt=0.05, walls=7,
              wall_sin=sins)
    init = lambda b: b.init_front(ns, [20.0] * len(ns))
    print(f"case resident segments {segment} orientation", flush=True)
    r, info, dr = segment_batch(S, [(10, 10, 120)] * len(ns), segment, [1, 2, 97, 300], init, **kw)
    assert info["kernel"] == S.KERNEL_RESIDENT and (info["segment"], info["halo"]) == segment
    t, dt_ = batch_fields(S, [(10, 10, 120)] * len(ns), "tiled", [1, 2, 97, 300], init, **kw)
    assert_bitwise(r, t)
    for a, b in zip(dr, dt_):
        assert a["interface_position"] == b["interface_position"] and a["step"] == 400


@pytest.mark.parametrize("walls", [1, 6])
def test_partly_walled_segments_equal_tiled(S, walls):
    """Walls on x only (the segments' x regions stop at the ghost layers) and on
    y and z only (the x regions wrap around a periodic axis while the y and z
    ghosts are refreshed inside every segment): 3 and 40 steps equal the tiled
    kernel bit for bit."""
    rng = np.random.default_rng(100 + walls)
    shapes = [(9, 7, 70), (6, 11, 45), (5, 5, 33)]
    ns, sins = [], []
    for _ in shapes:
        n = rng.normal(size=3)
        n[[d for d in range(3) if not (walls >> d) & 1]] = 0.0
        if walls & 1:
            n[0] = abs(n[0]) + 0.5
        n = n / np.linalg.norm(n)
        ns.append(n)
        sins.append(oracle.front_sin_alpha(n))
    kw = dict(lam=3.0, mu=0.03, stencil=26, coupling="local", dt=0.05, walls=walls, wall_sin=sins)
    init = lambda b: b.init_front(ns, [0.3, -0.2, 0.5])   # near the boxes' centres
    print(f"case resident segments walls={walls}", flush=True)
    r, info, _ = segment_batch(S, shapes, (6, 3), [3, 40], init, **kw)
    assert (info["segment"], info["halo"]) == (6, 3)
    t, _ = batch_fields(S, shapes, "tiled", [3, 40], init, **kw)
    assert_bitwise(r, t)
    for f in r[-1]:   # the fronts lie inside the boxes: neither phase fills them
        assert f.min() < 0.1 and f.max() > 0.9


@pytest.mark.parametrize("coupling,interp", [("local", "h3"), ("global", "h3"), ("cf", "h5")])
@pytest.mark.parametrize("segment", [(8, 4), (16, 16), (5, 2)])
def test_periodic_segments_equal_tiled(S, coupling, interp, segment):
    """Periodic slabs and ragged grids, some long enough to be cut (their
    segments' halos wrap around the x axis), some kept whole in the same launch:
    7 and 10 steps equal the tiled kernel bit for bit."""
    shapes = [(3, 3, 256), (3, 3, 64), (5, 4, 33), (7, 11, 9), (4, 6, 101)]
    hkl = [(1, 0, 0), (1, 1, 1), (2, 1, 1), (1, 2, 3), (3, 1, 0)]
    mu = 0.3 if coupling == "cf" else 0.04
    kw = dict(lam=2.5, mu=mu, stencil=26, coupling=coupling, interp=interp, u=(1.0, 2.0, 0.0), dt=0.02)
    init = lambda b: b.init_planar(hkl, [0.3, 0.1, 0.7, 0.2, 0.5])
    print(f"case resident segments {segment} periodic {coupling}+{interp}", flush=True)
    r, _, _ = segment_batch(S, shapes, segment, [7, 10], init, **kw)
    t, _ = batch_fields(S, shapes, "tiled", [7, 10], init, **kw)
    assert_bitwise(r, t)


def test_segments_over_many_launches_match_oracle(S):
    """Segments with a halo of 3 over 301 steps (101 launches, the last one
    step): within the FP32 bar of the oracle and equal to the tiled kernel."""
    shapes = [(4, 5, 90), (3, 3, 47)]
    lam, mu, steps = 3.0, 0.02, 301
    hkl = [(1, 0, 0), (2, 1, 0)]
    fields = [as_f32_input(oracle.init_planar(sh, h, 0.4, lam=lam)) for sh, h in zip(shapes, hkl)]
    ps = [oracle.params(sh, lam=lam, mu=mu, stencil=18, coupling="local", eps=1e-30) for sh in shapes]
    dt = min(stable_dt(p) for p in ps)
    kw = dict(lam=lam, mu=mu, stencil=18, coupling="local", dt=dt)
    def init(b):
        for i, f in enumerate(fields):
            b.set_field(i, f)
    print("case resident segments 301 steps", flush=True)
    r, info, _ = segment_batch(S, shapes, (7, 3), [steps], init, **kw)
    t, _ = batch_fields(S, shapes, "tiled", [steps], init, **kw)
    assert_bitwise(r, t)
    for i, p in enumerate(ps):
        p.dt = dt
        ref = oracle.step(p, fields[i], steps)
        assert float(np.abs(r[0][i].astype(np.float64) - ref).max()) <= 1e-5, i


def test_auto_picks_a_kernel_by_timing_and_equals_tiled(S):
    """Kernel AUTO on a batch of small grids times the tiled kernel, whole grids
    and x segments at the first step; whatever it keeps, the fields equal the
    tiled kernel's bit for bit, and the batch reports its choice."""
    shapes = [(10, 10, 120)] * 3 + [(3, 3, 256)] * 2
    hkl = [(1, 0, 0), (2, 1, 0), (1, 1, 1), (1, 0, 0), (3, 1, 1)]
    kw = dict(lam=4.0, mu=0.02, stencil=26, coupling="local", dt=0.05)
    init = lambda b: b.init_planar(hkl, [0.2, 0.4, 0.6, 0.1, 0.3])
    print("case resident auto", flush=True)
    a, info, _ = segment_batch(S, shapes, None, [50, 3], init, kernel="auto", **kw)
    print(f"  auto chose {info}", flush=True)
    assert info["kernel"] in (S.KERNEL_RESIDENT, S.KERNEL_TILED)
    if info["kernel"] == S.KERNEL_TILED:
        assert info["segment"] == 0 and info["halo"] == 0
    t, _ = batch_fields(S, shapes, "tiled", [50, 3], init, **kw)
    assert_bitwise(a, t)
