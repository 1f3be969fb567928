"""ctypes binding of libspfm.so (C ABI in include/spfm.h).

Argument marshalling only: every step of the SPFM time step runs in the HIP
kernels of the library.  PyTorch, when present, supplies device memory (the
two ping-pong buffers) and the stream the library orders its work on.  There
is no fallback: if the library has not been built the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspfm.so")

F32, F64 = 0, 1
LOCAL, GLOBAL, CF = 0, 1, 2
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_TILED, KERNEL_RESIDENT = 0, 1, 2, 3
_DTYPES = {"f32": F32, "float32": F32, "f64": F64, "float64": F64}
_COUPLINGS = {"local": LOCAL, "global": GLOBAL, "cf": CF}
_KERNELS = {"auto": KERNEL_AUTO, "plain": KERNEL_PLAIN, "tiled": KERNEL_TILED,
            "resident": KERNEL_RESIDENT}
_INTERPS = {"h3": 0, "h5": 1, "habel": 2}

OK, E_INVAL, E_NOMEM, E_HIP, E_UNSTABLE, E_DIVERGED, E_STATE = 0, -1, -2, -3, -4, -5, -6


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("coupling", ctypes.c_int32),
                ("u", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("gamma", ctypes.c_double * 3), ("C_Gamma", ctypes.c_double),
                ("eps", ctypes.c_double), ("tau", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("d_phi", ctypes.c_void_p * 2),
                ("kernel", ctypes.c_int32), ("allow_unstable", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("tsteps", ctypes.c_int32),
                ("walls", ctypes.c_int32), ("wall_sin", ctypes.c_double * 6),
                ("interp", ctypes.c_int32), ("conserve_volume", ctypes.c_int32),
                ("batch_wall_sin", ctypes.c_void_p), ("tile", ctypes.c_int32 * 2),
                ("segment", ctypes.c_int32 * 2)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time", ctypes.c_double),
                ("phase_volume", ctypes.c_double), ("interface_area", ctypes.c_double),
                ("interface_position", ctypes.c_double), ("velocity", ctypes.c_double),
                ("phi_min", ctypes.c_double), ("phi_max", ctypes.c_double),
                ("sum_phi", ctypes.c_double), ("sum_x", ctypes.c_double),
                ("diverged", ctypes.c_int32), ("mu", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("lam", "Gamma", "M", "mu", "dt", "dx", "C_Gamma", "eps", "tau")] + \
               [("gamma", ctypes.c_double * 3), ("dt_max", ctypes.c_double),
                ("stencil", ctypes.c_int32), ("coupling", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("tsteps", ctypes.c_int32),
                ("walls", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("conserve_volume", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("grids", ctypes.c_int32), ("points", ctypes.c_int64),
                ("segment", ctypes.c_int32), ("halo", ctypes.c_int32)]


class Contour(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double * 3), ("points", ctypes.c_int64),
                ("R_mean", ctypes.c_double), ("R_min", ctypes.c_double), ("R_max", ctypes.c_double),
                ("eps_eff", ctypes.c_double)]


class SpfmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"spfm status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libspfm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    sigs = {
        "spfm_create": ([ctypes.POINTER(Grid), d, d, d, d, ctypes.c_int, ctypes.POINTER(Options),
                         ctypes.POINTER(vp)], ctypes.c_int),
        "spfm_destroy": ([vp], None),
        "spfm_set_field": ([vp, vp, ctypes.c_int], ctypes.c_int),
        "spfm_get_field": ([vp, vp, ctypes.c_int], ctypes.c_int),
        "spfm_field_ptr": ([vp, ctypes.POINTER(vp)], ctypes.c_int),
        "spfm_init_planar": ([vp, ip, d], ctypes.c_int),
        "spfm_init_spheres": ([vp, i32, dp, dp], ctypes.c_int),
        "spfm_init_spheres_noalloc": ([vp, i32, dp, dp], ctypes.c_int),
        "spfm_init_front": ([vp, dp, d], ctypes.c_int),
        "spfm_init_box": ([vp, dp, dp], ctypes.c_int),
        "spfm_contour_stats": ([vp, ctypes.POINTER(Contour)], ctypes.c_int),
        "spfm_ray_radii": ([vp, dp, i32, dp, dp], ctypes.c_int),
        "spfm_energy": ([vp, ctypes.c_int, dp], ctypes.c_int),
        "spfm_set_mu": ([vp, d], ctypes.c_int),
        "spfm_force": ([vp, dp], ctypes.c_int),
        "spfm_step": ([vp, i64], ctypes.c_int),
        "spfm_diagnostics": ([vp, ctypes.POINTER(Diag)], ctypes.c_int),
        "spfm_get_info": ([vp, ctypes.POINTER(Info)], ctypes.c_int),
        "spfm_batch_create": ([i32, ctypes.POINTER(Grid), dp, dp, dp, dp, ctypes.c_int,
                               ctypes.POINTER(Options), ctypes.POINTER(vp)], ctypes.c_int),
        "spfm_batch_init_front": ([vp, dp, dp], ctypes.c_int),
        "spfm_batch_destroy": ([vp], None),
        "spfm_batch_init_planar": ([vp, ip, dp], ctypes.c_int),
        "spfm_batch_set_field": ([vp, i32, vp, ctypes.c_int], ctypes.c_int),
        "spfm_batch_get_field": ([vp, i32, vp, ctypes.c_int], ctypes.c_int),
        "spfm_batch_step": ([vp, i64], ctypes.c_int),
        "spfm_batch_diagnostics": ([vp, ctypes.POINTER(Diag)], ctypes.c_int),
        "spfm_batch_points": ([vp], i64),
        "spfm_batch_zchunk": ([vp], i32),
        "spfm_batch_kernel": ([vp], i32),
        "spfm_batch_get_info": ([vp, ctypes.POINTER(BatchInfo)], ctypes.c_int),
        "spfm_calibrate_cgamma": ([d, ctypes.c_int], d),
        "spfm_stable_dt": ([ctypes.c_int, ctypes.c_int, dp, dp, d, d, d, d, d, d], d),
        "spfm_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "spfm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st: int):
    if st != OK:
        L = load()
        raise SpfmError(st, (L.spfm_last_error() or b"").decode())


def _torch():
    try:
        import torch
        return torch
    except Exception:  # pragma: no cover - torch is part of the image
        return None


def _stream_handle(stream):
    if stream is None:
        torch = _torch()
        if torch is not None and torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _options(*, dtype="f32", coupling="local", u=(1.0, 0.0, 0.0), dt=None, gamma=None,
             C_Gamma=None, eps=None, tau=None, kernel="auto", stream=None,
             allow_unstable=False, zchunk=0, tsteps=0, walls=0, wall_sin=None,
             interp="h3", conserve_volume=False, tile=None, segment=None) -> Options:
    o = Options()
    o.dtype = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    o.coupling = _COUPLINGS[coupling] if isinstance(coupling, str) else int(coupling)
    o.u[:] = [float(v) for v in u]
    o.dt = float(dt) if dt else 0.0
    o.gamma[:] = [float(v) for v in gamma] if gamma is not None else [0.0, 0.0, 0.0]
    o.C_Gamma = float(C_Gamma) if C_Gamma else 0.0
    o.eps = float(eps) if eps else 0.0
    o.tau = float(tau) if tau else 0.0
    o.stream = _stream_handle(stream)
    o.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.allow_unstable = 1 if allow_unstable else 0
    o.zchunk = int(zchunk)
    o.tsteps = int(tsteps)
    o.walls = _walls_mask(walls)
    o.wall_sin[:] = [float(v) for v in wall_sin] if wall_sin is not None else [0.0] * 6
    o.interp = _INTERPS[interp] if isinstance(interp, str) else int(interp)
    o.conserve_volume = 1 if conserve_volume else 0
    o.tile[:] = [int(v) for v in tile] if tile is not None else [0, 0]
    o.segment[:] = [int(v) for v in segment] if segment is not None else [0, 0]
    return o


def _walls_mask(walls) -> int:
    """Walled axes as a bit mask: an int, or a string of axis letters ("xyz", "yz")."""
    if isinstance(walls, str):
        return sum(1 << "xyz".index(a) for a in set(walls))
    return int(walls)


def front_wall_sin(n):
    """Face values (-x, +x, -y, +y, -z, +z) of wall_sin that hold a planar front
    of normal n (into phase 0) exactly: n . e over the outward face normals."""
    v = np.asarray(n, dtype=np.float64)
    v = v / np.linalg.norm(v)
    return (-v[0], v[0], -v[1], v[1], -v[2], v[2])


def _np_dtype(code: int):
    return np.float64 if code == F64 else np.float32


class Spfm:
    """One periodic grid of shape (nz, ny, nx) stepped by the HIP library."""

    def __init__(self, shape: Sequence[int], *, dx: float = 1.0, lam: float = 4.0,
                 Gamma: float = 1.0, M: float = 1.0, mu: float = 0.0, stencil: int = 26,
                 torch_buffers: bool = True, **opts):
        L = load()
        nz, ny, nx = (int(v) for v in shape)
        self.shape = (nz, ny, nx)
        self._opts = _options(**opts)
        self.np_dtype = _np_dtype(self._opts.dtype)
        self._buffers = None
        torch = _torch()
        w = self._opts.walls
        self.stored_shape = (nz + 2 * ((w >> 2) & 1), ny + 2 * ((w >> 1) & 1), nx + 2 * (w & 1))
        if torch_buffers and torch is not None and torch.cuda.is_available():
            tdt = torch.float64 if self._opts.dtype == F64 else torch.float32
            self._buffers = [torch.zeros(self.stored_shape, dtype=tdt, device="cuda")
                             for _ in range(2)]
            self._opts.d_phi[0] = self._buffers[0].data_ptr()
            self._opts.d_phi[1] = self._buffers[1].data_ptr()
        g = Grid(nx, ny, nz, float(dx))
        h = ctypes.c_void_p()
        _check(L.spfm_create(ctypes.byref(g), float(lam), float(Gamma), float(M), float(mu),
                             int(stencil), ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None):
            load().spfm_destroy(self._h)
            self._h = None
        self._buffers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- field --
    def set_field(self, field):
        torch = _torch()
        if torch is not None and isinstance(field, torch.Tensor):
            assert tuple(field.shape) == self.shape and field.is_contiguous()
            assert field.dtype == (torch.float64 if self.np_dtype == np.float64 else torch.float32)
            _check(load().spfm_set_field(self._h, field.data_ptr(), 1 if field.is_cuda else 0))
            return
        a = np.ascontiguousarray(field, dtype=self.np_dtype)
        assert a.shape == self.shape, (a.shape, self.shape)
        _check(load().spfm_set_field(self._h, a.ctypes.data, 0))

    def get_field(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.np_dtype)
        _check(load().spfm_get_field(self._h, out.ctypes.data, 0))
        return out

    def field_ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(load().spfm_field_ptr(self._h, ctypes.byref(p)))
        return int(p.value)

    def init_planar(self, hkl, offset: float = 0.0):
        h = (ctypes.c_int32 * 3)(*[int(v) for v in hkl])
        _check(load().spfm_init_planar(self._h, h, float(offset)))

    def init_spheres(self, centers, radii, noalloc: bool = False):
        """Eq. 3 grains; noalloc: through spfm_init_spheres_noalloc (no device
        allocation, at most 4096 spheres)."""
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        assert c.shape[0] == r.size
        dp = ctypes.POINTER(ctypes.c_double)
        f = load().spfm_init_spheres_noalloc if noalloc else load().spfm_init_spheres
        _check(f(self._h, r.size, c.ctypes.data_as(dp), r.ctypes.data_as(dp)))

    def init_box(self, lo, hi):
        a = np.ascontiguousarray(lo, dtype=np.float64).reshape(3)
        b = np.ascontiguousarray(hi, dtype=np.float64).reshape(3)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().spfm_init_box(self._h, a.ctypes.data_as(dp), b.ctypes.data_as(dp)))

    def contour_stats(self) -> dict:
        c = Contour()
        _check(load().spfm_contour_stats(self._h, ctypes.byref(c)))
        out = {n: getattr(c, n) for n, _ in Contour._fields_}
        out["centre"] = tuple(c.centre)
        return out

    def energy(self, with_mu: bool = False) -> float:
        """Free energy of Eq. 1 of the current field (with mu h(phi) if with_mu)."""
        out = ctypes.c_double()
        _check(load().spfm_energy(self._h, 1 if with_mu else 0, ctypes.byref(out)))
        return out.value

    def ray_radii(self, dirs, centre=None) -> np.ndarray:
        """Radii of the phi = 1/2 surface along the rays `dirs` (n x 3) from
        `centre` (default: the barycentre of contour_stats)."""
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        c = np.ascontiguousarray(np.asarray(centre if centre is not None
                                            else self.contour_stats()["centre"], dtype=np.float64))
        out = np.empty(d.shape[0])
        dptr = ctypes.POINTER(ctypes.c_double)
        _check(load().spfm_ray_radii(self._h, c.ctypes.data_as(dptr), int(d.shape[0]),
                                     d.ctypes.data_as(dptr), out.ctypes.data_as(dptr)))
        return out

    def init_front(self, n, offset: float = 0.0):
        v = np.ascontiguousarray(n, dtype=np.float64).reshape(3)
        _check(load().spfm_init_front(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      float(offset)))

    # -- stepping --
    def force(self) -> float:
        """Total force of the current field: the system sum of the Eq. 4 bracket."""
        v = ctypes.c_double()
        _check(load().spfm_force(self._h, ctypes.byref(v)))
        return float(v.value)

    def set_mu(self, mu: float):
        _check(load().spfm_set_mu(self._h, float(mu)))

    def step(self, n: int = 1):
        _check(load().spfm_step(self._h, int(n)))

    def diagnostics(self) -> dict:
        d = Diag()
        _check(load().spfm_diagnostics(self._h, ctypes.byref(d)))
        return d.as_dict()

    def info(self) -> dict:
        i = Info()
        _check(load().spfm_get_info(self._h, ctypes.byref(i)))
        out = {n: getattr(i, n) for n, _ in Info._fields_}
        out["gamma"] = tuple(i.gamma)
        return out


class SpfmBatch:
    """Many independent grids stepped by one launch per step.  With walls,
    wall_sin may hold one row of six face values per grid."""

    def __init__(self, shapes, *, lam, mu, dx=1.0, Gamma=1.0, M=1.0, stencil=26, wall_sin=None,
                 **opts):
        L = load()
        n = len(shapes)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        per_grid = wall_sin is not None and np.ndim(wall_sin) == 2
        if per_grid:
            self._wall_sin = np.ascontiguousarray(np.asarray(wall_sin, dtype=np.float64).reshape(n, 6))
        elif wall_sin is not None:
            opts["wall_sin"] = wall_sin

        def arr(v):
            v = np.broadcast_to(np.asarray(v, dtype=np.float64), (n,))
            return np.ascontiguousarray(v)
        self._lam, self._mu = arr(lam), arr(mu)
        self._Gamma, self._M = arr(Gamma), arr(M)
        dxs = arr(dx)
        grids = (Grid * n)(*[Grid(s[2], s[1], s[0], float(dxs[i])) for i, s in enumerate(self.shapes)])
        self._opts = _options(**opts)
        if per_grid:
            self._opts.batch_wall_sin = self._wall_sin.ctypes.data
        dp = ctypes.POINTER(ctypes.c_double)
        h = ctypes.c_void_p()
        _check(L.spfm_batch_create(n, grids, self._lam.ctypes.data_as(dp), self._Gamma.ctypes.data_as(dp),
                                   self._M.ctypes.data_as(dp), self._mu.ctypes.data_as(dp),
                                   int(stencil), ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            load().spfm_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def points(self) -> int:
        return int(load().spfm_batch_points(self._h))

    @property
    def zchunk(self) -> int:
        """Leading z-chunk of the work items (chosen at the first step with kernel="auto")."""
        return int(load().spfm_batch_zchunk(self._h))

    @property
    def kernel(self) -> str:
        """The step kernel in use: "tiled" or "resident"."""
        return {KERNEL_TILED: "tiled", KERNEL_RESIDENT: "resident"}[int(load().spfm_batch_kernel(self._h))]

    def info(self) -> dict:
        """Kernel, tile column and z-chunk in use (after tuning), grid and point counts."""
        i = BatchInfo()
        _check(load().spfm_batch_get_info(self._h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in BatchInfo._fields_}

    def init_planar(self, hkls, offsets):
        h = np.ascontiguousarray(np.asarray(hkls, dtype=np.int32).reshape(-1, 3))
        o = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1))
        _check(load().spfm_batch_init_planar(self._h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             o.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def init_front(self, normals, offsets):
        """Planar fronts of the given normals (one row of three per grid)."""
        nv = np.ascontiguousarray(np.asarray(normals, dtype=np.float64).reshape(-1, 3))
        o = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().spfm_batch_init_front(self._h, nv.ctypes.data_as(dp), o.ctypes.data_as(dp)))

    def set_field(self, i: int, field):
        a = np.ascontiguousarray(field, dtype=np.float32)
        assert a.shape == self.shapes[i]
        _check(load().spfm_batch_set_field(self._h, int(i), a.ctypes.data, 0))

    def get_field(self, i: int) -> np.ndarray:
        out = np.empty(self.shapes[i], dtype=np.float32)
        _check(load().spfm_batch_get_field(self._h, int(i), out.ctypes.data, 0))
        return out

    def step(self, n: int = 1):
        _check(load().spfm_batch_step(self._h, int(n)))

    def diagnostics(self):
        d = (Diag * self.n)()
        _check(load().spfm_batch_diagnostics(self._h, d))
        return [x.as_dict() for x in d]


def calibrate_cgamma(lam_over_dx: float, coupling="local") -> float:
    c = _COUPLINGS[coupling] if isinstance(coupling, str) else int(coupling)
    return float(load().spfm_calibrate_cgamma(float(lam_over_dx), c))


def stable_dt(stencil, coupling, u, gamma, lam, Gamma, M, mu, dx, C_Gamma=0.0) -> float:
    c = _COUPLINGS[coupling] if isinstance(coupling, str) else int(coupling)
    uu = (ctypes.c_double * 3)(*u)
    gg = (ctypes.c_double * 3)(*(gamma if gamma is not None else (0.0, 0.0, 0.0)))
    return float(load().spfm_stable_dt(int(stencil), c, uu, gg, float(lam), float(Gamma), float(M),
                                       float(mu), float(dx), float(C_Gamma)))


def try_create(shape, **kw):
    """spfm_create without allocating: returns (status, message).  Used to
    exercise argument validation, which happens before any HIP call."""
    L = load()
    nz, ny, nx = shape
    dx = kw.pop("dx", 1.0)
    lam = kw.pop("lam", 4.0)
    Gamma = kw.pop("Gamma", 1.0)
    M = kw.pop("M", 1.0)
    mu = kw.pop("mu", 0.0)
    stencil = kw.pop("stencil", 26)
    o = _options(stream=0, **kw)
    g = Grid(nx, ny, nz, dx)
    h = ctypes.c_void_p()
    st = L.spfm_create(ctypes.byref(g), lam, Gamma, M, mu, stencil, ctypes.byref(o), ctypes.byref(h))
    if st == OK:
        L.spfm_destroy(h)
    return st, (L.spfm_last_error() or b"").decode()
