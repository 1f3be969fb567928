"""GPU parity of the temporally blocked step (tsteps steps fused per pass).

Every fused level evaluates the single-step tiled sweep's point update on the
same per-plane sums, so n fused steps must equal n tiled steps bit for bit;
the tiled kernel itself is held to the oracle in test_gpu_parity.  Runs whose
length is not a multiple of tsteps finish with single tiled steps and are held
to the oracle (max |dphi| <= 1e-5, FP32 against FP64)."""
import numpy as np
import pytest

import oracle
from gpu_common import as_f32_input, noisy_field, slab111, sphere12, stable_dt
from paper_1910_05180_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_05180_amd import spfm
    spfm.load()
    return spfm


def run(S, phi0, steps, *, lam, mu, stencil, coupling, dt, C_Gamma, stream=None, **kw):
    with S.Spfm(phi0.shape, lam=lam, mu=mu, stencil=stencil, coupling=coupling, u=(1.0, 2.0, 0.0),
                dt=dt, C_Gamma=C_Gamma, stream=stream, **kw) as s:
        s.set_field(phi0.astype(np.float32))
        s.step(steps)
        if stream is not None:
            stream.synchronize()
        return s.get_field()


def fused_vs_tiled(S, phi0, tsteps, steps, *, lam=1.5, mu=0.01, stencil=26, coupling="local",
                   zchunk=0, stream=None):
    p = oracle.params(phi0.shape, lam=lam, mu=mu, stencil=stencil, coupling=coupling,
                      u=(1.0, 2.0, 0.0))
    dt = stable_dt(p)
    print(f"case shape={phi0.shape} tsteps={tsteps} steps={steps} S={stencil} {coupling} "
          f"zchunk={zchunk} graph={stream is not None}", flush=True)
    common = dict(lam=lam, mu=mu, stencil=stencil, coupling=coupling, dt=dt, C_Gamma=p.C_Gamma)
    ref = run(S, phi0, steps, kernel="tiled", **common)
    got = run(S, phi0, steps, kernel="tiled", tsteps=tsteps, zchunk=zchunk, stream=stream, **common)
    return got, ref


@pytest.mark.parametrize("tsteps", [2, 3, 4])
@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
def test_fused_equals_tiled_bitwise(S, tsteps, coupling):
    got, ref = fused_vs_tiled(S, slab111(), tsteps, 6 * tsteps, coupling=coupling)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("stencil", [6, 18])
@pytest.mark.parametrize("coupling", ["local", "global", "cf"])
def test_fused_equals_tiled_small_stencils(S, stencil, coupling):
    got, ref = fused_vs_tiled(S, slab111(), 2, 10, stencil=stencil, coupling=coupling)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("zchunk", [1, 3, 7, 64])
def test_fused_grain_any_zchunk(S, zchunk):
    """A grain (the TI_n normal varies in every direction) and z-chunks that
    split the sweep unevenly, down to one plane per block."""
    got, ref = fused_vs_tiled(S, sphere12(), 3, 12, lam=2.0, mu=0.0, zchunk=zchunk)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (7, 3, 130), (33, 4, 65), (5, 70, 9)])
def test_fused_small_and_ragged_grids(S, shape):
    """Footprints wider than the grid wrap around it several times."""
    phi0 = as_f32_input(noisy_field(shape, 3.0, 11))
    for tsteps in (2, 4):
        got, ref = fused_vs_tiled(S, phi0, tsteps, 2 * tsteps, lam=3.0, mu=0.02)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), tsteps


def test_fused_graph_replay(S):
    """Captured HIP graphs of fused launches (stream given, many steps)."""
    import torch
    st = torch.cuda.Stream()
    got, ref = fused_vs_tiled(S, slab111(), 2, 2 * 2 * 16 + 6, stream=st)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("tsteps,steps", [(2, 7), (3, 11), (4, 6)])
def test_remainder_steps_match_oracle(S, tsteps, steps):
    """n not a multiple of tsteps: fused launches then single tiled steps."""
    phi0 = as_f32_input(slab111())
    p = oracle.params(phi0.shape, lam=1.5, mu=0.01, stencil=26, coupling="local")
    p.dt = stable_dt(p)
    ref = oracle.step(p, phi0, steps)
    with S.Spfm(phi0.shape, lam=1.5, mu=0.01, stencil=26, dt=p.dt, C_Gamma=p.C_Gamma,
                kernel="tiled", tsteps=tsteps) as s:
        s.set_field(phi0)
        s.step(steps)
        d = s.diagnostics()
        got = s.get_field().astype(np.float64)
        assert s.info()["tsteps"] == tsteps
    assert d["step"] == steps
    assert float(np.abs(got - ref).max()) <= 1e-5


def test_fused_grains512_bitwise_in_bench_configuration(S):
    """The 512^3 grain workload at full size: 2 fused launches of 2 steps
    against 4 single tiled steps, every point compared, for TI_n and CF."""
    import torch
    w = inputs.grains512()
    st = torch.cuda.Stream()
    for coupling in ("local", "cf"):
        fields = []
        for kw in (dict(kernel="tiled", zchunk=32), dict(kernel="tiled", tsteps=2, zchunk=64)):
            print(f"case grains512 {coupling} {kw}", flush=True)
            with torch.cuda.stream(st):
                with S.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, coupling=coupling, stream=st,
                            **kw) as s:
                    s.init_spheres(w.centers, w.radii)
                    s.step(4)
                    st.synchronize()
                    fields.append(s.get_field())
        assert np.array_equal(fields[0].view(np.uint32), fields[1].view(np.uint32)), coupling
