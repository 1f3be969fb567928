"""Seeded workload generators: determinism and the published SplitMix64 stream."""
import math

from paper_1910_05180_amd import inputs as I


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 from state 0 (Steele, Lea & Flood 2014).
    r = I.SplitMix64(0)
    assert r.next_u64() == 0xE220A8397B1DCDAF
    assert r.next_u64() == 0x6E789E6AA1B965F4


def test_uniform_range_and_determinism():
    a, b = I.SplitMix64(42), I.SplitMix64(42)
    xs = [a.uniform() for _ in range(1000)]
    assert xs == [b.uniform() for _ in range(1000)]
    assert all(0.0 <= x < 1.0 for x in xs)


def test_workloads():
    p = I.planar32()
    assert p.shape == (32, 32, 32) and 0.0 <= p.offset < 1.0 and p.stencil == 6
    sweep = I.planar128_mu_sweep()
    assert len(sweep) == 16 and abs(sweep[0].mu + 0.1) < 1e-15 and abs(sweep[-1].mu - 0.1) < 1e-15
    b = I.batch64()
    assert len(b) == 64
    assert all(q.shape[0] in (48, 64, 96, 128, 160) and q.hkl != (0, 0, 0) for q in b)
    assert all(3.0 <= q.lam <= 6.0 and -0.1 <= q.mu <= 0.1 for q in b)
    s = I.sphere256()
    assert len(s.rays) == 1000
    assert all(abs(math.sqrt(sum(c * c for c in v)) - 1) < 1e-12 for v in s.rays)


def test_grains_do_not_overlap():
    g = I.grains512(count=60)
    L = g.shape[0]
    for i in range(len(g.radii)):
        for j in range(i):
            d2 = 0.0
            for a in range(3):
                d = g.centers[i][a] - g.centers[j][a]
                d -= L * round(d / L)
                d2 += d * d
            assert math.sqrt(d2) >= g.radii[i] + g.radii[j] + 2 * g.lam
