"""Tile shapes of the tiled kernels and their autotuner: every compiled shape
computes the same per-plane sums and point update, so a step's result does
not depend on the shape (nor on the z-chunk) bit for bit; the tuned choice is
reported by spfm_get_info / spfm_batch_get_info."""
import numpy as np
import pytest

import oracle
from gpu_common import sphere12, slab111, stable_dt

pytestmark = pytest.mark.gpu

F32_SHAPES = [(16, 8), (32, 8), (64, 8), (16, 16), (32, 16), (64, 16)]
F64_LOCAL_SHAPES = [(64, 8), (32, 8), (16, 8)]


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def run(S, phi0, steps, **kw):
    with S.Spfm(phi0.shape, **kw) as s:
        s.set_field(phi0)
        s.step(steps)
        return s.get_field(), s.info()


@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
@pytest.mark.parametrize("stencil", [6, 26])
def test_fp32_shapes_equal_bitwise(S, coupling, stencil):
    """A grain in a 70 x 37 x 45 box: ragged against every shape along x and y."""
    phi0 = sphere12(2.0)
    p = oracle.params(phi0.shape, lam=2.0, mu=0.01, stencil=stencil, coupling=coupling, u=(1.0, 2.0, 0.0))
    kw = dict(lam=2.0, mu=0.01, stencil=stencil, dtype="f32", coupling=coupling, u=(1.0, 2.0, 0.0),
              dt=stable_dt(p), kernel="tiled")
    ref, info = run(S, phi0, 9, **kw)
    assert (info["tile_x"], info["tile_y"]) == ((16, 8) if coupling == "local" else (64, 8))
    for shape in F32_SHAPES:
        print(f"case tile {shape} {coupling} S={stencil}", flush=True)
        got, info = run(S, phi0, 9, tile=shape, **kw)
        assert (info["tile_x"], info["tile_y"]) == shape
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), shape


def test_fp64_local_shapes_equal_bitwise(S):
    phi0 = slab111(3.0)
    kw = dict(lam=3.0, mu=0.02, stencil=26, dtype="f64", coupling="local", kernel="tiled")
    ref, _ = run(S, phi0, 7, **kw)
    for shape in F64_LOCAL_SHAPES:
        print(f"case f64 tile {shape}", flush=True)
        got, info = run(S, phi0, 7, tile=shape, **kw)
        assert (info["tile_x"], info["tile_y"]) == shape
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), shape


def test_fp32_wide_tiles_match_oracle(S):
    """The widest and tallest shapes against the oracle (FP32 bar), 60 steps."""
    phi0 = sphere12(2.0)
    ref_in = phi0.astype(np.float32).astype(np.float64)
    p = oracle.params(phi0.shape, lam=2.0, mu=0.0, stencil=26, coupling="local", eps=1e-30)
    ref = oracle.step(p, ref_in, 60)
    for shape in [(64, 16), (32, 16)]:
        got, _ = run(S, phi0, 60, lam=2.0, mu=0.0, stencil=26, dtype="f32", coupling="local",
                     kernel="tiled", tile=shape, eps=1e-30, C_Gamma=p.C_Gamma)
        assert float(np.abs(got.astype(np.float64) - ref).max()) <= 1e-5, shape


def test_autotuned_context_reports_its_choice_and_equals_default(S):
    """Kernel AUTO on a grid that fills the GPU times every compiled (shape,
    z-chunk) pair at the first step; whatever it picks, the field equals the
    untuned default bit for bit."""
    shape = (128, 128, 128)
    phi0 = oracle.init_spheres(shape, [(64.3, 63.7, 64.1)], [40.0], lam=4.0)
    kw = dict(lam=4.0, mu=0.0, stencil=26, dtype="f32", coupling="local")
    ref, info0 = run(S, phi0, 10, kernel="tiled", **kw)
    got, info = run(S, phi0, 10, kernel="auto", **kw)
    print(f"tuned tile {info['tile_x']}x{info['tile_y']} zchunk {info['zchunk']}", flush=True)
    assert (info["tile_x"], info["tile_y"]) in F32_SHAPES
    assert info["zchunk"] in (8, 16, 32, 64)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("tile", [(16, 8), (64, 8), (32, 16)])
def test_batch_shapes_equal_bitwise(S, tile):
    """A batch of uneven slabs with explicit tiles equals the default tile."""
    shapes = [(48, 48, 48), (33, 40, 29), (20, 64, 70)]
    hkl = [(1, 2, 3), (2, -1, 1), (0, 1, 4)]
    kw = dict(lam=[4.0, 3.5, 5.0], mu=[0.05, -0.03, 0.01], stencil=26, coupling="local", kernel="tiled")
    out = []
    for t in (None, tile):
        with S.SpfmBatch(shapes, tile=t, **kw) as b:
            b.init_planar(hkl, [0.1, 0.6, 0.3])
            b.step(11)
            info = b.info()
            out.append([b.get_field(i) for i in range(len(shapes))])
        assert (info["tile_x"], info["tile_y"]) == (tile if t else (16, 8))
        assert info["kernel"] == S.KERNEL_TILED and info["grids"] == 3
    for a, b_ in zip(*out):
        assert np.array_equal(a.view(np.uint32), b_.view(np.uint32))
