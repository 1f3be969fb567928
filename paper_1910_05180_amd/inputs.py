"""Seeded synthetic workloads for the SPFM step.

This module draws only the *parameters* of the synthetic workloads (offsets,
normals, radii, centres, widths, driving forces) from a SplitMix64 stream; it
contains none of the method's arithmetic.  Both the GPU path and the CPU oracle
build their fields from these parameters with their own code.

SplitMix64 follows Steele, Lea & Flood, "Fast splittable pseudorandom number
generators" (OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the two
xor-shift-multiply rounds of the published finaliser.  Doubles are
(x >> 11) * 2^-53 in [0, 1).

The paper measures on synthetic ideal-profile set-ups only (planar interfaces
of Sec. 3.1-3.2, a relaxing particle in Sec. 3.3); the workloads below stand in
for those at the sizes the throughput study uses.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

BASE_SEED = 1910051800
_MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        span = hi - lo + 1
        return lo + int(self.uniform() * span)


@dataclass
class Planar:
    """Periodic slab with integer normal hkl (see the planar initial field)."""
    shape: Tuple[int, int, int]   # (nz, ny, nx)
    hkl: Tuple[int, int, int]
    offset: float                 # shift of the slab centre along the normal, in dx
    lam: float
    mu: float
    dx: float = 1.0
    Gamma: float = 1.0
    M: float = 1.0
    dt: float = 0.1
    stencil: int = 26
    steps: int = 0


@dataclass
class Spheres:
    shape: Tuple[int, int, int]
    centers: List[Tuple[float, float, float]]
    radii: List[float]
    lam: float
    mu: float
    dx: float = 1.0
    Gamma: float = 1.0
    M: float = 1.0
    dt: float = 0.1
    stencil: int = 26
    steps: int = 0
    rays: List[Tuple[float, float, float]] = field(default_factory=list)


def planar32(seed: int = BASE_SEED + 0) -> Planar:
    """32^3 periodic [100] slab, lambda = 4 dx, mu = 0.05, 6 neighbours, 500 steps;
    slab centre at the box centre plus an offset drawn from U[0, 1) dx."""
    r = SplitMix64(seed)
    return Planar(shape=(32, 32, 32), hkl=(1, 0, 0), offset=r.uniform(), lam=4.0, mu=0.05,
                  stencil=6, steps=500)


def planar128_mu_sweep(seed: int = BASE_SEED + 1) -> List[Planar]:
    """128^3 periodic slab with normal (1,2,3), lambda = 5 dx, 26 neighbours,
    16 driving forces evenly spaced in [-0.1, 0.1], 2000 steps each."""
    r = SplitMix64(seed)
    off = r.uniform()
    return [Planar(shape=(128, 128, 128), hkl=(1, 2, 3), offset=off, lam=5.0,
                   mu=-0.1 + 0.2 * i / 15.0, stencil=26, steps=2000) for i in range(16)]


def sphere256(mu: float = 0.0, seed: int = BASE_SEED + 2, nrays: int = 1000) -> Spheres:
    """256^3 box, one grain of radius 60 dx at (128,128,128), lambda = 4 dx,
    26 neighbours, 5000 steps; nrays directions uniform on the unit sphere
    (z ~ U[-1,1], azimuth ~ U[0, 2 pi)) for the isotropy measure."""
    r = SplitMix64(seed)
    rays = []
    for _ in range(nrays):
        zc = r.uniform_range(-1.0, 1.0)
        az = r.uniform_range(0.0, 2.0 * math.pi)
        s = math.sqrt(max(0.0, 1.0 - zc * zc))
        rays.append((s * math.cos(az), s * math.sin(az), zc))
    return Spheres(shape=(256, 256, 256), centers=[(128.0, 128.0, 128.0)], radii=[60.0],
                   lam=4.0, mu=mu, stencil=26, steps=5000, rays=rays)


def batch64(seed: int = BASE_SEED + 3, count: int = 64) -> List[Planar]:
    """count independent periodic slabs: cube edge from {48,64,96,128,160},
    integer normal with components in [-4, 4] (not all zero), lambda ~ U[3, 6] dx,
    mu ~ U[-0.1, 0.1], offset ~ U[0, 1) dx, 26 neighbours, 3000 steps."""
    r = SplitMix64(seed)
    edges = (48, 64, 96, 128, 160)
    out = []
    for _ in range(count):
        L = edges[r.randint(0, 4)]
        while True:
            hkl = (r.randint(-4, 4), r.randint(-4, 4), r.randint(-4, 4))
            if hkl != (0, 0, 0):
                break
        lam = r.uniform_range(3.0, 6.0)
        mu = r.uniform_range(-0.1, 0.1)
        off = r.uniform()
        out.append(Planar(shape=(L, L, L), hkl=hkl, offset=off, lam=lam, mu=mu, stencil=26,
                          steps=3000))
    return out


def grains512(seed: int = BASE_SEED + 4, count: int = 300, edge: int = 512,
              lam: float = 4.0) -> Spheres:
    """edge^3 box with count non-overlapping grains, radii ~ U[8, 30] dx, centres
    ~ U[0, edge)^3, rejected unless every periodic centre distance is at least
    R_i + R_j + 2 lambda; mu = 0.01, 26 neighbours, 2000 steps."""
    r = SplitMix64(seed)
    centers: List[Tuple[float, float, float]] = []
    radii: List[float] = []
    tries = 0
    while len(centers) < count:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place grains")
        R = r.uniform_range(8.0, 30.0)
        c = (r.uniform() * edge, r.uniform() * edge, r.uniform() * edge)
        ok = True
        for cc, RR in zip(centers, radii):
            d2 = 0.0
            for a in range(3):
                d = c[a] - cc[a]
                d -= edge * round(d / edge)
                d2 += d * d
            if d2 < (R + RR + 2.0 * lam) ** 2:
                ok = False
                break
        if ok:
            centers.append(c)
            radii.append(R)
    return Spheres(shape=(edge, edge, edge), centers=centers, radii=radii, lam=lam, mu=0.01,
                   stencil=26, steps=2000)


def grains_twin(seed: int = BASE_SEED + 4, edge: int = 128) -> Spheres:
    """The grain workload at a 128^3 twin: the grain count scaled by volume."""
    count = max(1, round(300 * (edge / 512.0) ** 3))
    return grains512(seed=seed, count=count, edge=edge)
