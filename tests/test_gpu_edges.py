"""Degenerate and extreme cases of the step API on the device: zero steps,
one-grid batches, z-chunks of one plane and of the whole grid, and batches
that mix the smallest grid with large ones.  The step's result never depends
on how the work is cut, so these compare library paths bit for bit; the mixed
batch is also held to the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import as_f32_input, noisy_field, slab111, sphere12, stable_dt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_zero_steps_change_nothing(S, dtype):
    phi0 = slab111(3.0)
    print(f"case zero steps {dtype}", flush=True)
    with S.Spfm(phi0.shape, lam=3.0, mu=0.02, stencil=26, dtype=dtype, kernel="tiled") as s:
        s.set_field(phi0)
        before = s.get_field()
        s.step(0)
        d = s.diagnostics()
        after = s.get_field()
    assert d["step"] == 0
    assert np.array_equal(before, after)


@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
@pytest.mark.parametrize("zchunk", [1, 4096])
def test_extreme_zchunks_equal_the_default(S, coupling, zchunk):
    """One plane per block, and one block per tile column (zchunk above nz)."""
    phi0 = sphere12(2.0)
    p = oracle.params(phi0.shape, lam=2.0, mu=0.01, stencil=26, coupling=coupling, u=(1.0, 2.0, 0.0))
    dt = stable_dt(p)
    out = []
    for zc in (0, zchunk):
        print(f"case zchunk={zc} {coupling}", flush=True)
        with S.Spfm(phi0.shape, lam=2.0, mu=0.01, stencil=26, dtype="f32", coupling=coupling,
                    u=(1.0, 2.0, 0.0), dt=dt, kernel="tiled", zchunk=zc) as s:
            s.set_field(phi0)
            s.step(12)
            out.append(s.get_field())
    assert np.array_equal(out[0].view(np.uint32), out[1].view(np.uint32))


def test_fp64_whole_column_blocks_equal_the_default(S):
    phi0 = slab111(3.0)
    out = []
    for zc in (0, 4096):
        with S.Spfm(phi0.shape, lam=3.0, mu=0.02, stencil=26, dtype="f64", kernel="tiled",
                    zchunk=zc) as s:
            s.set_field(phi0)
            s.step(10)
            out.append(s.get_field())
    assert np.array_equal(out[0].view(np.uint64), out[1].view(np.uint64))


@pytest.mark.parametrize("coupling", ["local", "cf"])
def test_one_grid_batch_equals_the_context(S, coupling):
    phi0 = as_f32_input(sphere12(2.0))
    p = oracle.params(phi0.shape, lam=2.0, mu=0.01, stencil=26, coupling=coupling)
    dt = stable_dt(p)
    print(f"case one-grid batch {coupling}", flush=True)
    with S.SpfmBatch([phi0.shape], lam=2.0, mu=0.01, stencil=26, coupling=coupling, dt=dt) as b:
        b.set_field(0, phi0)
        b.step(20)
        got = b.get_field(0)
    with S.Spfm(phi0.shape, lam=2.0, mu=0.01, stencil=26, dtype="f32", coupling=coupling, dt=dt,
                kernel="tiled") as s:
        s.set_field(phi0)
        s.step(20)
        ref = s.get_field()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_batch_mixing_the_smallest_grid_with_large_ones(S):
    """A 3^3 grid (every halo wraps onto itself) beside grids of several tiles,
    each grid bitwise equal to its own context and within 1e-5 of the oracle."""
    shapes = [(3, 3, 3), (40, 33, 70), (5, 70, 9), (3, 3, 3), (33, 4, 65)]
    lam, mu = 3.0, 0.02
    fields = [as_f32_input(noisy_field(sh, lam, 21 + i)) for i, sh in enumerate(shapes)]
    ps = [oracle.params(sh, lam=lam, mu=mu, stencil=26, coupling="local", eps=1e-30) for sh in shapes]
    dt = min(stable_dt(p) for p in ps)
    steps = 4
    print(f"case mixed batch {shapes}", flush=True)
    with S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling="local", dt=dt) as b:
        for i, f in enumerate(fields):
            b.set_field(i, f)
        b.step(steps)
        got = [b.get_field(i) for i in range(len(shapes))]
    for i, sh in enumerate(shapes):
        with S.Spfm(sh, lam=lam, mu=mu, stencil=26, dtype="f32", coupling="local", dt=dt,
                    kernel="tiled") as s:
            s.set_field(fields[i])
            s.step(steps)
            single = s.get_field()
        assert np.array_equal(got[i].view(np.uint32), single.view(np.uint32)), i
        ps[i].dt = dt
        ref = oracle.step(ps[i], fields[i], steps)
        assert float(np.abs(got[i].astype(np.float64) - ref).max()) <= 1e-5, i


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-6)])
@pytest.mark.parametrize("op", ["swap_xy", "swap_xz", "reflect_x", "reflect_yz"])
def test_cubic_symmetry_on_the_device(S, dtype, tol, op):
    """A cubic rotation or reflection of the input permutes the output (the
    oracle's symmetry pin, on the device).  The kernels add neighbour pairs in
    a fixed order, so the result agrees to rounding, not bit for bit."""
    lam = 3.0
    shape = (36, 36, 36)   # cube: the axis swaps keep the shape
    phi0 = oracle.init_spheres(shape, [(14.3, 19.1, 16.7)], [8.5], lam=lam)
    if dtype == "f32":
        phi0 = as_f32_input(phi0)
    ops = {"swap_xy": lambda a: np.ascontiguousarray(np.swapaxes(a, 1, 2)),
           "swap_xz": lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 2)),
           "reflect_x": lambda a: np.ascontiguousarray(a[:, :, ::-1]),
           "reflect_yz": lambda a: np.ascontiguousarray(a[::-1, ::-1, :])}
    T = ops[op]
    eps = 1e-300 if dtype == "f64" else 1e-30
    out = []
    for f in (phi0, T(phi0)):
        with S.Spfm(shape, lam=lam, mu=0.01, stencil=26, dtype=dtype, coupling="local", eps=eps,
                    kernel="tiled") as s:
            s.set_field(f)
            s.step(10)
            out.append(s.get_field().astype(np.float64))
    assert float(np.abs(T(out[0]) - out[1]).max()) <= tol


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_set_mu_between_graph_replays(S, dtype, tol):
    """Steps on a non-null stream replay captured graphs of 16 launches; set_mu
    waits for them, drops the graphs and the next steps use the new driving
    force.  The oracle runs the same switch (Eq. 2 with mu, then with mu')."""
    import torch
    phi0 = slab111(3.0)
    eps = 1e-300 if dtype == "f64" else 1e-30
    start = phi0 if dtype == "f64" else as_f32_input(phi0)
    ref = start
    for mu in (0.04, -0.06):
        p = oracle.params(phi0.shape, lam=3.0, mu=mu, dt=0.1, stencil=26, coupling="local", eps=eps)
        ref = oracle.step(p, ref, 40)
    stream = torch.cuda.Stream()
    print(f"case set_mu between graph replays {dtype}", flush=True)
    with S.Spfm(phi0.shape, lam=3.0, mu=0.04, stencil=26, dtype=dtype, coupling="local", dt=0.1,
                kernel="tiled", stream=stream, eps=eps, C_Gamma=p.C_Gamma) as s:
        s.set_field(phi0)
        s.step(40)          # two graph replays and 8 single launches
        s.set_mu(-0.06)
        s.step(40)
        d = s.diagnostics()
        got = s.get_field().astype(np.float64)
    assert d["step"] == 80 and d["mu"] == -0.06
    err = float(np.abs(got - ref).max())
    print(f"  max|dphi| = {err:.3e}", flush=True)
    assert err <= tol
