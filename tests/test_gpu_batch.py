"""Batched stepping of many uneven periodic grids in one launch per step."""
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


def small_batch():
    """Five slabs of different sizes, widths, driving forces and normals; each
    box is compatible with its normal so that P >= 6 lambda."""
    return [
        dict(shape=(20, 24, 70), hkl=(1, 0, 0), lam=3.0, mu=0.05, off=0.2),
        dict(shape=(33, 17, 40), hkl=(0, 0, 1), lam=2.5, mu=-0.04, off=0.7),
        dict(shape=(48, 48, 48), hkl=(1, 1, 0), lam=3.5, mu=0.02, off=0.1),
        dict(shape=(16, 64, 64), hkl=(1, 1, 0), lam=2.2, mu=0.08, off=0.9),
        dict(shape=(36, 36, 36), hkl=(1, 0, 1), lam=2.0, mu=-0.01, off=0.5),
    ]


def test_batch_equals_single_grids_and_oracle(S):
    cases = small_batch()
    steps = 120
    shapes = [c["shape"] for c in cases]
    lam = [c["lam"] for c in cases]
    mu = [c["mu"] for c in cases]
    b = S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling="local")
    fields = [oracle.init_planar(c["shape"], c["hkl"], c["off"], lam=c["lam"]) for c in cases]
    for i, f in enumerate(fields):
        b.set_field(i, f)
    b.step(steps)
    for i, c in enumerate(cases):
        print(f"batch instance {i} {c}", flush=True)
        got = b.get_field(i)
        with S.Spfm(c["shape"], lam=c["lam"], mu=c["mu"], stencil=26, dtype="f32",
                    coupling="local", kernel="tiled") as s:
            s.set_field(fields[i])
            s.step(steps)
            single = s.get_field()
        assert np.array_equal(got, single), i
        p = oracle.params(c["shape"], lam=c["lam"], mu=c["mu"], stencil=26, coupling="local",
                          eps=1e-30)
        ref = oracle.step(p, as_f32_input(fields[i]), steps)
        assert np.abs(got.astype(np.float64) - ref).max() <= 1e-5, i
    b.close()


def test_batch_init_and_diagnostics(S):
    cases = small_batch()
    b = S.SpfmBatch([c["shape"] for c in cases], lam=[c["lam"] for c in cases],
                    mu=[c["mu"] for c in cases], stencil=26)
    assert b.points == sum(int(np.prod(c["shape"])) for c in cases)
    b.init_planar([c["hkl"] for c in cases], [c["off"] for c in cases])
    d0 = b.diagnostics()
    for i, c in enumerate(cases):
        ref = oracle.init_planar(c["shape"], c["hkl"], c["off"], lam=c["lam"])
        got = b.get_field(i).astype(np.float64)
        assert np.abs(got - ref).max() < 6e-8
        s1, _ = oracle.exact_sums(got)
        assert d0[i]["sum_phi"] == pytest.approx(s1, rel=1e-15)
        assert d0[i]["interface_position"] == 0.0
    b.step(400)
    d1 = b.diagnostics()
    for i, c in enumerate(cases):
        v = d1[i]["interface_position"] / d1[i]["time"]
        assert abs(v / -c["mu"] - 1) < 2e-2, (i, v)
    b.close()


def test_full_batch_prefix_matches_single_grids(S):
    """The 64-grid workload (edges 48..160): every grid of the batch equals the
    single-grid tiled kernel bitwise after a 100-step prefix."""
    from paper_1910_05180_amd import inputs
    ws = inputs.batch64()
    steps = 100
    b = S.SpfmBatch([w.shape for w in ws], lam=[w.lam for w in ws], mu=[w.mu for w in ws],
                    stencil=26)
    b.init_planar([w.hkl for w in ws], [w.offset for w in ws])
    b.step(steps)
    for i in range(0, len(ws), 7):
        w = ws[i]
        print(f"full batch instance {i} shape={w.shape} hkl={w.hkl}", flush=True)
        with S.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, dtype="f32", kernel="tiled") as s:
            s.init_planar(w.hkl, w.offset)
            s.step(steps)
            single = s.get_field()
        assert np.array_equal(b.get_field(i), single), i
    b.close()


def test_batch_zchunk_choice_does_not_change_results(S):
    """kernel="auto" times z-chunks of 4..64 planes at the first step and keeps
    the fastest; an explicit zchunk is kept as given; kernel="tiled" takes the
    size rule (this small batch gives too few threads for 32-plane chunks).  The
    fields after the same steps are bitwise equal whatever was chosen."""
    cases = small_batch()
    shapes = [c["shape"] for c in cases]
    lam = [c["lam"] for c in cases]
    mu = [c["mu"] for c in cases]
    fields = [oracle.init_planar(c["shape"], c["hkl"], c["off"], lam=c["lam"]) for c in cases]
    out, chosen = {}, {}
    for name, opts in [("auto", dict(kernel="auto")), ("tiled", dict(kernel="tiled")),
                       ("auto_z7", dict(kernel="auto", zchunk=7)), ("z32", dict(kernel="tiled", zchunk=32))]:
        print(f"case batch {name}", flush=True)
        with S.SpfmBatch(shapes, lam=lam, mu=mu, stencil=26, coupling="local", **opts) as b:
            for i, f in enumerate(fields):
                b.set_field(i, f)
            b.step(30)
            chosen[name] = b.zchunk
            out[name] = [b.get_field(i) for i in range(len(cases))]
    assert chosen["auto"] in (2, 4, 8, 16, 32, 64)
    assert chosen["auto_z7"] == 7 and chosen["z32"] == 32
    assert chosen["tiled"] in (2, 4)   # 278824 points: 32 planes would give 2^16 threads
    for name in ("tiled", "auto_z7", "z32"):
        for i in range(len(cases)):
            assert np.array_equal(out[name][i], out["auto"][i]), (name, i)


def test_full_batch_instances_match_oracle(S):
    """The 64-grid workload from the oracle's own FP32-rounded initial fields:
    after 100 steps the 8 smallest grids (edges 48 and 64, where the FP64 oracle
    finishes in seconds) are within 1e-5 of the oracle."""
    from paper_1910_05180_amd import inputs
    ws = inputs.batch64()
    steps = 100
    fields = [as_f32_input(oracle.init_planar(w.shape, w.hkl, w.offset, lam=w.lam)) for w in ws]
    with S.SpfmBatch([w.shape for w in ws], lam=[w.lam for w in ws], mu=[w.mu for w in ws],
                     stencil=26, coupling="local") as b:
        for i, f in enumerate(fields):
            b.set_field(i, f)
        b.step(steps)
        picks = sorted(range(len(ws)), key=lambda i: (np.prod(ws[i].shape), i))[:8]
        got = {i: b.get_field(i).astype(np.float64) for i in picks}
    for i in picks:
        w = ws[i]
        print(f"batch64 instance {i} shape={w.shape} hkl={w.hkl} lam={w.lam:.3f} mu={w.mu:+.4f}",
              flush=True)
        p = oracle.params(w.shape, lam=w.lam, mu=w.mu, stencil=26, coupling="local", eps=1e-30)
        ref = oracle.step(p, fields[i], steps)
        assert float(np.abs(got[i] - ref).max()) <= 1e-5, i


def test_grids_beyond_32_bit_element_offsets(S):
    """Two grids with the largest accepted z-plane (3 x 16384 x 32767 each,
    3.2e9 points together) ahead of two small ones, so the small grids start
    beyond 2^31 elements (2^33 bytes) into the batch buffers: after 20 steps
    each small grid equals a single-grid context bit for bit."""
    big = (3, 16384, 32767)
    cases = [dict(shape=big, hkl=(1, 0, 0), lam=4.0, mu=0.02, off=0.3),
             dict(shape=big, hkl=(0, 1, 0), lam=4.0, mu=-0.02, off=0.6),
             dict(shape=(40, 36, 52), hkl=(0, 0, 1), lam=3.0, mu=0.03, off=0.2),
             dict(shape=(33, 17, 40), hkl=(0, 0, 1), lam=2.5, mu=-0.04, off=0.7)]
    steps = 20
    with S.SpfmBatch([c["shape"] for c in cases], lam=[c["lam"] for c in cases],
                     mu=[c["mu"] for c in cases], stencil=26, kernel="tiled") as b:
        b.init_planar([c["hkl"] for c in cases], [c["off"] for c in cases])
        b.step(steps)
        got = {i: b.get_field(i) for i in (2, 3)}
    for i in (2, 3):
        c = cases[i]
        print(f"batch beyond 2^31 elements: instance {i} {c}", flush=True)
        with S.Spfm(c["shape"], lam=c["lam"], mu=c["mu"], stencil=26, dtype="f32",
                    kernel="tiled") as s:
            s.init_planar(c["hkl"], c["off"])
            s.step(steps)
            assert np.array_equal(got[i], s.get_field()), i
