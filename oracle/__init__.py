"""CPU FP64 oracle of the Sharp Phase-Field Method (arXiv:1910.05180).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does, and
the two share no code.  This module only marshals numpy arrays into the plain C
library ``spfm_oracle.c`` (which holds every equation) and adds exact
(``math.fsum``) reductions for the diagnostics of Sec. 2.3 and Sec. 3.

Field arrays are numpy float64 of shape (nz, ny, nx), x fastest, periodic.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spfm_oracle.c")
_SO = os.path.join(_HERE, "libspfm_oracle.so")
_lock = threading.Lock()
_lib = None

LOCAL, GLOBAL, CF = 0, 1, 2
COUPLINGS = {"local": LOCAL, "global": GLOBAL, "cf": CF}
H3, H5, HABEL = 0, 1, 2
INTERPS = {"h3": H3, "h5": H5, "habel": HABEL}


def build() -> str:
    """Compile the oracle with gcc (plain C, OpenMP over z planes)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-std=c11", "-D_DEFAULT_SOURCE", "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("lam", ctypes.c_double), ("Gamma", ctypes.c_double),
        ("M", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
        ("C_Gamma", ctypes.c_double), ("stencil", ctypes.c_int), ("coupling", ctypes.c_int),
        ("u", ctypes.c_double * 3), ("gamma", ctypes.c_double * 3),
        ("eps", ctypes.c_double), ("tau", ctypes.c_double),
        ("interp", ctypes.c_int),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_SO)
            dp = ctypes.POINTER(ctypes.c_double)
            pp = ctypes.POINTER(Params)
            L.orc_direction.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
            L.orc_direction.restype = ctypes.c_int
            L.orc_nu.argtypes = [ctypes.c_int]
            L.orc_nu.restype = ctypes.c_double
            for f in (L.orc_g, L.orc_g_prime):
                f.argtypes = [ctypes.c_double] * 4
                f.restype = ctypes.c_double
            L.orc_normal.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
            L.orc_rate.argtypes = [pp, dp, dp]
            L.orc_rate_points.argtypes = [pp, dp, ctypes.c_long, ctypes.POINTER(ctypes.c_long), dp]
            L.orc_step.argtypes = [pp, dp, ctypes.c_long]
            L.orc_step.restype = ctypes.c_int
            L.orc_energy.argtypes = [pp, dp, ctypes.c_int]
            L.orc_energy.restype = ctypes.c_double
            L.orc_calibrate_cgamma.argtypes = [ctypes.c_double]
            L.orc_calibrate_cgamma.restype = ctypes.c_double
            L.orc_stable_dt.argtypes = [pp]
            L.orc_stable_dt.restype = ctypes.c_double
            L.orc_init_planar.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double,
                                                               ctypes.POINTER(ctypes.c_int),
                                                               ctypes.c_double, dp]
            L.orc_init_spheres.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double,
                                                               ctypes.c_int, dp, dp, dp]
            L.orc_spheres_at.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double,
                                                              ctypes.c_int, dp, dp, ctypes.c_long,
                                                              ctypes.POINTER(ctypes.c_int), dp]
            for f in (L.orc_interp, L.orc_interp_prime):
                f.argtypes = [ctypes.c_int, ctypes.c_double]
                f.restype = ctypes.c_double
            L.orc_wall_value.argtypes = [ctypes.c_double, ctypes.c_double]
            L.orc_wall_value.restype = ctypes.c_double
            L.orc_fill_walls.argtypes = [pp, ctypes.c_int, dp, dp]
            L.orc_step_walls.argtypes = [pp, ctypes.c_int, dp, dp, ctypes.c_long]
            L.orc_step_walls.restype = ctypes.c_int
            L.orc_init_front.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, dp,
                                                              ctypes.c_double, dp]
            L.orc_step_constant_volume.argtypes = [pp, dp, ctypes.c_long, dp]
            L.orc_step_constant_volume.restype = ctypes.c_int
            L.orc_init_box.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, dp, dp, dp]
            L.orc_contour_points.argtypes = [pp, dp, ctypes.c_long, dp]
            L.orc_contour_points.restype = ctypes.c_long
            L.orc_num_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_gamma(stencil: int):
    """Shell weights (reading): the leading-order isotropic shell combinations
    of Sec. 2.1's three Laplacian realisations; gamma_1 = 1 - gamma_2 - gamma_3."""
    return {6: (1.0, 0.0, 0.0), 18: (1.0 / 3.0, 2.0 / 3.0, 0.0),
            26: (14.0 / 30.0, 12.0 / 30.0, 4.0 / 30.0)}[stencil]


def params(shape, *, dx=1.0, lam=4.0, Gamma=1.0, M=1.0, mu=0.0, dt=0.1, stencil=26,
           coupling="local", u=(1.0, 0.0, 0.0), gamma=None, C_Gamma=None, eps=1e-12,
           tau=1e-3, interp="h3") -> Params:
    nz, ny, nx = shape
    p = Params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.dx, p.lam, p.Gamma, p.M, p.mu, p.dt = dx, lam, Gamma, M, mu, dt
    p.stencil = stencil
    p.coupling = COUPLINGS[coupling] if isinstance(coupling, str) else int(coupling)
    p.u[:] = u
    p.gamma[:] = default_gamma(stencil) if gamma is None else gamma
    if C_Gamma is None:
        C_Gamma = 2.0 / 3.0 if p.coupling == CF else calibrate_cgamma(lam / dx)
    p.C_Gamma = C_Gamma
    p.eps, p.tau = eps, tau
    p.interp = INTERPS[interp] if isinstance(interp, str) else int(interp)
    return p


def direction(k: int):
    r = (ctypes.c_int * 3)()
    shell = lib().orc_direction(k, r)
    return (r[0], r[1], r[2]), shell


def nu(shell: int) -> float:
    return lib().orc_nu(shell)


def g(phi: float, a: float, rho: float, lam: float) -> float:
    return lib().orc_g(phi, a, rho, lam)


def g_prime(phi: float, a: float, rho: float, lam: float) -> float:
    return lib().orc_g_prime(phi, a, rho, lam)


def _check(p: Params, phi: np.ndarray):
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    assert phi.shape == (p.nz, p.ny, p.nx), (phi.shape, (p.nz, p.ny, p.nx))


def normal(p: Params, phi: np.ndarray, x: int, y: int, z: int):
    _check(p, phi)
    n = np.zeros(3)
    lib().orc_normal(ctypes.byref(p), _dp(phi), x, y, z, _dp(n))
    return n


def rate(p: Params, phi: np.ndarray) -> np.ndarray:
    _check(p, phi)
    out = np.empty_like(phi)
    lib().orc_rate(ctypes.byref(p), _dp(phi), _dp(out))
    return out


def rate_points(p: Params, phi: np.ndarray, idx: np.ndarray) -> np.ndarray:
    _check(p, phi)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size)
    lib().orc_rate_points(ctypes.byref(p), _dp(phi), idx.size,
                          idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out))
    return out


def step(p: Params, phi: np.ndarray, nsteps: int) -> np.ndarray:
    out = np.array(phi, dtype=np.float64, order="C", copy=True)
    _check(p, out)
    if lib().orc_step(ctypes.byref(p), _dp(out), int(nsteps)) != 0:
        raise MemoryError("oracle step allocation failed")
    return out


def energy(p: Params, phi: np.ndarray, with_mu: bool = False) -> float:
    _check(p, phi)
    return lib().orc_energy(ctypes.byref(p), _dp(phi), 1 if with_mu else 0)


def calibrate_cgamma(lam_over_dx: float) -> float:
    return lib().orc_calibrate_cgamma(float(lam_over_dx))


def stable_dt(p: Params) -> float:
    return lib().orc_stable_dt(ctypes.byref(p))


def init_planar(shape, hkl, offset, *, dx=1.0, lam=4.0) -> np.ndarray:
    nz, ny, nx = shape
    out = np.empty(shape, dtype=np.float64)
    h = (ctypes.c_int * 3)(*hkl)
    lib().orc_init_planar(nx, ny, nz, dx, lam, h, float(offset), _dp(out))
    return out


def init_spheres(shape, centers, radii, *, dx=1.0, lam=4.0) -> np.ndarray:
    nz, ny, nx = shape
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    out = np.empty(shape, dtype=np.float64)
    lib().orc_init_spheres(nx, ny, nz, dx, lam, r.size, _dp(c), _dp(r), _dp(out))
    return out


def spheres_at(shape, centers, radii, xyz, *, dx=1.0, lam=4.0) -> np.ndarray:
    """The init_spheres field of a box of `shape` at integer coordinates xyz (N x 3, x y z)."""
    nz, ny, nx = shape
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    q = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.empty(q.shape[0])
    lib().orc_spheres_at(nx, ny, nz, dx, lam, r.size, _dp(c), _dp(r), q.shape[0],
                         q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out))
    return out


def cone_step(p: Params, shape, field_at, centres_xyz, nsteps: int) -> np.ndarray:
    """Values after nsteps steps at the given points of a large periodic box, each
    from its dependency cone: a point's value after K steps depends only on the
    (2K+1)^3 box around it, so the oracle steps that crop (built by
    field_at(xyz) with periodic coordinates) and keeps its centre."""
    nz, ny, nx = shape
    k = int(nsteps)
    w = 2 * k + 1
    off = np.arange(-k, k + 1)
    dz, dy, dxx = np.meshgrid(off, off, off, indexing="ij")
    out = np.empty(len(centres_xyz))
    q = Params()
    ctypes.pointer(q)[0] = p
    q.nx = q.ny = q.nz = w
    for i, (x, y, z) in enumerate(centres_xyz):
        xyz = np.stack([(x + dxx) % nx, (y + dy) % ny, (z + dz) % nz], axis=-1).reshape(-1, 3)
        crop = field_at(xyz).reshape(w, w, w)
        out[i] = step(q, crop, k)[k, k, k] if k > 0 else crop[0, 0, 0]
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------------------
# Walls with a contact angle (Sec. 2.2, Eq. 7).  A walled axis d (bit d of
# `walls`) has one ghost layer at each end; sin_alpha[2d] and [2d+1] belong to
# the low and high face of axis d and are n . e of the front normal n the wall
# imposes, e the outward normal of the face.
# ---------------------------------------------------------------------------
def interp(which, phi: float) -> float:
    """Interpolation function h of Tab. 2 ("h3", "h5", "habel")."""
    w = INTERPS[which] if isinstance(which, str) else int(which)
    return lib().orc_interp(w, float(phi))


def interp_prime(which, phi: float) -> float:
    w = INTERPS[which] if isinstance(which, str) else int(which)
    return lib().orc_interp_prime(w, float(phi))


def step_constant_volume(p: Params, phi: np.ndarray, nsteps: int):
    """nsteps forward-Euler steps with the driving force chosen at every step so
    that sum phi stays constant (Sec. 3.3).  Returns (phi, mu per step)."""
    _check(p, phi)
    out = phi.copy()
    mu = np.empty(int(nsteps))
    if lib().orc_step_constant_volume(ctypes.byref(p), _dp(out), int(nsteps), _dp(mu)) != 0:
        raise MemoryError("oracle step allocation failed")
    return out, mu


def init_box(shape, lo, hi, *, dx=1.0, lam=4.0) -> np.ndarray:
    """Box particle with smooth faces (product of Eq. 3 top hats over the axes)."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=np.float64)
    a = np.ascontiguousarray(lo, dtype=np.float64)
    b = np.ascontiguousarray(hi, dtype=np.float64)
    lib().orc_init_box(nx, ny, nz, dx, lam, _dp(a), _dp(b), _dp(out))
    return out


def contour_points(p: Params, phi: np.ndarray) -> np.ndarray:
    """phi = 1/2 contour points (x, y, z) on the grid edges (Eq. 8-10, l = 1/2)."""
    _check(p, phi)
    n = lib().orc_contour_points(ctypes.byref(p), _dp(phi), 0, None)
    pts = np.empty((max(n, 1), 3))
    lib().orc_contour_points(ctypes.byref(p), _dp(phi), n, _dp(pts))
    return pts[:n]


def sphericity(p: Params, phi: np.ndarray):
    """Residual anisotropy of a particle (Sec. 3.3): barycentre c = sum phi x / sum phi,
    R_i = |contour point - c|, eps_eff = (R_max - R_min) / (2 R_mean).
    Returns (eps_eff, R_mean, R_min, R_max, c, number of points)."""
    nz, ny, nx = phi.shape
    w = math.fsum(phi.ravel())
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.array([math.fsum((phi * xx).ravel()), math.fsum((phi * yy).ravel()),
                  math.fsum((phi * zz).ravel())]) / w * p.dx
    pts = contour_points(p, phi)
    R = np.sqrt(((pts - c) ** 2).sum(axis=1))
    Rm = math.fsum(R) / R.size
    return (R.max() - R.min()) / (2 * Rm), Rm, R.min(), R.max(), c, R.size


def ray_radii(phi: np.ndarray, centre, rays, *, dx: float = 1.0, eps: float = 1e-12,
              step: float = 0.25, bisections: int = 44) -> np.ndarray:
    """Radii of a particle's phi = 1/2 surface along seeded rays from `centre`
    (the isotropy measure along rays of the 256^3 grain configuration; the
    particle shape of Sec. 3.3 sampled along directions).  psi = ln((1-phi)/phi)
    (the inverse of Eq. 3 up to the factor lambda/4, which does not move its
    zero), phi clamped to [eps, 1-eps], is interpolated trilinearly between grid
    points of the periodic box.  Each ray is marched in steps of `step` grid
    spacings from the centre to the first sample with psi >= 0, and that step is
    bisected `bisections` times (0.25 / 2^44 < 1e-13).  NaN where a ray runs half
    the smallest box edge without crossing or starts outside.  centre and radii
    in units of length (dx times grid index)."""
    nz, ny, nx = phi.shape
    f = np.clip(np.asarray(phi, dtype=np.float64), eps, 1.0 - eps)
    psi = np.log((1.0 - f) / f)
    d = np.asarray(rays, dtype=np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1)[:, None]
    c = np.asarray(centre, dtype=np.float64) / dx

    def sample(t, sel=slice(None)):
        q = c[None, :] + t[:, None] * d[sel]
        i0 = np.floor(q)
        w = q - i0
        ix, iy, iz = (i0[:, 0].astype(np.int64), i0[:, 1].astype(np.int64), i0[:, 2].astype(np.int64))
        val = np.zeros(t.shape)
        for dz in (0, 1):
            wz = w[:, 2] if dz else 1.0 - w[:, 2]
            for dy in (0, 1):
                wy = w[:, 1] if dy else 1.0 - w[:, 1]
                for dxx in (0, 1):
                    wx = w[:, 0] if dxx else 1.0 - w[:, 0]
                    val += wz * wy * wx * psi[(iz + dz) % nz, (iy + dy) % ny, (ix + dxx) % nx]
        return val

    n = d.shape[0]
    kmax = int(math.floor(0.5 * min(nx, ny, nz) / step))
    hi = np.full(n, np.nan)
    inside = sample(np.zeros(n)) < 0.0
    todo = inside.copy()
    for k in range(1, kmax + 1):
        if not todo.any():
            break
        t = np.full(n, k * step)
        out = todo & (sample(t) >= 0.0)
        hi[out] = k * step
        todo &= ~out
    ok = ~np.isnan(hi)
    a, b = hi - step, hi.copy()
    for _ in range(bisections):
        m = 0.5 * (a + b)
        pos = np.zeros(n, dtype=bool)
        pos[ok] = sample(m[ok], ok) >= 0.0
        b = np.where(ok & pos, m, b)
        a = np.where(ok & ~pos, m, a)
    r = 0.5 * (a + b) * dx
    r[~ok] = np.nan
    return r


def wall_value(phi_in: float, a: float) -> float:
    return lib().orc_wall_value(float(phi_in), float(a))


def front(shape, n, offset=0.0, *, dx=1.0, lam=4.0) -> np.ndarray:
    """Single planar front of Eq. 3 with normal n (into phase 0) through the box
    centre shifted by offset along n, on the points of `shape`."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=np.float64)
    nv = np.ascontiguousarray(n, dtype=np.float64)
    lib().orc_init_front(nx, ny, nz, dx, lam, _dp(nv), float(offset), _dp(out))
    return out


def front_sin_alpha(n):
    """The six face values that hold a planar front of normal n exactly."""
    v = np.asarray(n, dtype=np.float64)
    v = v / np.linalg.norm(v)
    return [-v[0], v[0], -v[1], v[1], -v[2], v[2]]


def padded_shape(shape, walls: int):
    nz, ny, nx = shape
    return (nz + 2 * ((walls >> 2) & 1), ny + 2 * ((walls >> 1) & 1), nx + 2 * (walls & 1))


def interior(phi_padded: np.ndarray, walls: int) -> np.ndarray:
    gz, gy, gx = (walls >> 2) & 1, (walls >> 1) & 1, walls & 1
    nz, ny, nx = phi_padded.shape
    return phi_padded[gz:nz - gz, gy:ny - gy, gx:nx - gx]


def pad(phi: np.ndarray, walls: int) -> np.ndarray:
    """Copy of phi with zero ghost layers on the walled axes."""
    out = np.zeros(padded_shape(phi.shape, walls))
    interior(out, walls)[...] = phi
    return out


def _padded_params(p: Params, walls: int) -> Params:
    q = Params()
    ctypes.memmove(ctypes.byref(q), ctypes.byref(p), ctypes.sizeof(Params))
    q.nz, q.ny, q.nx = padded_shape((p.nz, p.ny, p.nx), walls)
    return q


def fill_walls(p: Params, phi_padded: np.ndarray, walls: int, sin_alpha) -> np.ndarray:
    """Fill the ghost layers of phi_padded in place; p holds the interior shape."""
    q = _padded_params(p, walls)
    _check(q, phi_padded)
    sa = np.ascontiguousarray(sin_alpha, dtype=np.float64)
    lib().orc_fill_walls(ctypes.byref(q), int(walls), _dp(sa), _dp(phi_padded))
    return phi_padded


def step_walls(p: Params, phi: np.ndarray, walls: int, sin_alpha, nsteps: int,
               padded: bool = False) -> np.ndarray:
    """nsteps forward-Euler steps of the interior field phi (shape of p) between
    contact-angle walls; returns the interior (or the filled padded field)."""
    q = _padded_params(p, walls)
    work = pad(np.asarray(phi, dtype=np.float64), walls)
    sa = np.ascontiguousarray(sin_alpha, dtype=np.float64)
    if lib().orc_step_walls(ctypes.byref(q), int(walls), _dp(sa), _dp(work), int(nsteps)) != 0:
        raise MemoryError("oracle step allocation failed")
    return work if padded else interior(work, walls).copy()


def rate_walls(p: Params, phi: np.ndarray, walls: int, sin_alpha) -> np.ndarray:
    """d phi / dt of Eq. 2 at the interior points, with the walls filled."""
    q = _padded_params(p, walls)
    work = fill_walls(p, pad(np.asarray(phi, dtype=np.float64), walls), walls, sin_alpha)
    return interior(rate(q, work), walls).copy()


# ---------------------------------------------------------------------------
# Diagnostics (exact sums).  The paper plots interface position and velocity
# (Fig. 1b) but defines neither from the field; the readings used here:
#   phase volume     V1 = dx^3 sum phi
#   interface area   A_if = (4/lambda) dx^3 sum phi (1 - phi)   (exact for an
#                    ideal planar profile: the integral of phi(1-phi) across it
#                    is lambda/4)
#   slab position    delta(t) = (V1(t) - V1(0)) / A_tot, A_tot = 2 L^2 |N| / gcd(N)
#   sphere radius    R_V with (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16) = V1
# ---------------------------------------------------------------------------

def exact_sums(phi: np.ndarray):
    """Exactly rounded sums of phi and phi(1 - phi) (FP64 per element)."""
    a = np.asarray(phi, dtype=np.float64).ravel()
    return math.fsum(a.tolist()), math.fsum((a * (1.0 - a)).tolist())


def phase_volume(phi: np.ndarray, dx: float = 1.0) -> float:
    return exact_sums(phi)[0] * dx ** 3


def interface_area(phi: np.ndarray, lam: float, dx: float = 1.0) -> float:
    return 4.0 / lam * exact_sums(phi)[1] * dx ** 3


def slab_area(shape, hkl, dx: float = 1.0) -> float:
    """Total interface area of the periodic slab of orc_init_planar."""
    nz, ny, nx = shape
    nn = math.sqrt(sum(h * h for h in hkl))
    gg = 0
    for n_i, h in zip((nx, ny, nz), hkl):
        gg = math.gcd(gg, abs(n_i * h))
    P = gg * dx / nn
    return 2.0 * nx * ny * nz * dx ** 3 / P


def sphere_radius_from_volume(V1: float, lam: float) -> float:
    """Solve (4 pi/3)(R^3 + R pi^2 lambda^2/16) = V1 for R by Newton's method."""
    c = math.pi ** 2 * lam ** 2 / 16.0
    R = (3.0 * V1 / (4.0 * math.pi)) ** (1.0 / 3.0)
    for _ in range(60):
        f = 4.0 * math.pi / 3.0 * (R ** 3 + R * c) - V1
        d = 4.0 * math.pi / 3.0 * (3.0 * R * R + c)
        R -= f / d
    return R
