"""The allocation-free sphere initialisation (spfm_init_spheres_noalloc) against
spfm_init_spheres through the C ABI: the same field bit for bit, on two calls
in a row whose second has fewer spheres (the static device table keeps the
first call's entries beyond the second's count, which must not leak in), for
FP32 and FP64, periodic and walled grids; sizes beyond the table are refused."""
import ctypes

import numpy as np
import pytest

from paper_1910_05180_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def both(S, shape, centers, radii, **kw):
    out = []
    for noalloc in (False, True):
        with S.Spfm(shape, lam=4.0, stencil=26, kernel="tiled", **kw) as s:
            s.init_spheres(centers, radii, noalloc=noalloc)
            d = s.diagnostics()
            out.append((s.get_field(), d))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_equals_allocating_init_on_two_calls(S, dtype):
    w = inputs.grains_twin()            # 5 grains in 128^3
    big = inputs.grains512(count=300)   # 300 grain centres of the 512^3 workload
    shape = (64, 80, 96)
    # first call: 300 spheres (scaled into the box), second: the 5 of the twin
    c300 = [(x * 96 / 512, y * 80 / 512, z * 64 / 512) for (x, y, z) in big.centers]
    r300 = [r * 0.3 for r in big.radii]
    c5 = [(x * 96 / 128, y * 80 / 128, z * 64 / 128) for (x, y, z) in w.centers]
    r5 = [r * 0.6 for r in w.radii]
    with S.Spfm(shape, lam=2.0, stencil=26, dtype=dtype, kernel="tiled") as a, \
            S.Spfm(shape, lam=2.0, stencil=26, dtype=dtype, kernel="tiled") as b:
        for cc, rr in ((c300, r300), (c5, r5)):
            print(f"case noalloc {dtype} n={len(rr)}", flush=True)
            a.init_spheres(cc, rr)
            b.init_spheres(cc, rr, noalloc=True)
            fa, fb = a.get_field(), b.get_field()
            assert np.array_equal(fa.view(np.uint8), fb.view(np.uint8))
            assert fb.max() > 0.9 and fb.min() < 1e-2
            da, db = a.diagnostics(), b.diagnostics()
            assert da["sum_phi"] == db["sum_phi"]


def test_noalloc_single_grain_tracks_radius_and_walled_grid(S):
    """One sphere: the interface position is the volume radius, as for the
    allocating call; a walled grid fills its interior the same way."""
    f = both(S, (40, 44, 48), [(20.3, 21.7, 19.2)], [9.0], dtype="f32")
    assert np.array_equal(f[0][0], f[1][0])
    assert f[0][1]["interface_position"] == f[1][1]["interface_position"]
    g = both(S, (12, 14, 16), [(6.0, 7.0, 8.0)], [4.0], dtype="f64", walls="xz")
    assert np.array_equal(g[0][0], g[1][0])


def test_noalloc_rejects_too_many_and_bad_lists(S):
    L = S.load()
    with S.Spfm((8, 8, 8), lam=4.0, stencil=26, kernel="tiled") as s:
        n = 4097
        c = np.zeros((n, 3))
        r = np.ones(n)
        dp = ctypes.POINTER(ctypes.c_double)
        st = L.spfm_init_spheres_noalloc(s._h, n, c.ctypes.data_as(dp), r.ctypes.data_as(dp))
        assert st == S.E_INVAL
        assert b"4096" in L.spfm_last_error()
        st = L.spfm_init_spheres_noalloc(s._h, -1, c.ctypes.data_as(dp), r.ctypes.data_as(dp))
        assert st == S.E_INVAL
        r[0] = np.nan
        st = L.spfm_init_spheres_noalloc(s._h, 2, c.ctypes.data_as(dp), r.ctypes.data_as(dp))
        assert st == S.E_INVAL
        # zero spheres: an empty field
        s.init_spheres(np.zeros((0, 3)), np.zeros(0), noalloc=True)
        assert np.all(s.get_field() == 0)
