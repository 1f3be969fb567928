"""Throughput of the SPFM explicit step on one MI355X.

Headline: FP32, 26 neighbours, TI_n (local normal), tiled HIP kernel on the
256^3 periodic grain workload (one grain of radius 60 dx at the box centre,
lambda = 4 dx, mu = 0, Gamma = M = dx = 1, dt = 0.1), in GLUPS (10^9 lattice
point updates per second) and as a fraction of the HBM roofline.  Beside it:
the plain per-grid FP64 kernel on the same workload, and the CPU oracle timed
on a bounded sample of it on the host cores.

Prints one JSON line.  Only one GPU is used: --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ALG_BYTES_F32 = 8              # read phi^n + write phi^{n+1} per point per step
ALG_BYTES_F64 = 16
# FP32 VALU issue peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz lane-operations per second (one FP32 add, mul, fma, compare, select
# or transcendental per lane per cycle).  A secondary figure: the step is
# priced against the HBM roof, as the metric asks.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic FP32 operations per point update of the TI_n 26-neighbour step,
# counted from the per-point formulas the kernel evaluates, by the class of the
# point: 28 where phi(1-phi) = 0 (psi' 6, plane sums 6, shell sums 8, update 7,
# test 1), 64 in the tail branch (plus the normal 9, the exponentials and c_i
# 15, the tail sums 9, u and its term 2, test 1) and 157 with the full coupling
# (93 more: 2 sinh 6, x-scaled terms 4, the shell-2 and shell-3 y_k 40, three
# running fractions 39, their sum 3, select 1).  The mix is measured on the
# field at the start and the end of the timed window.
OPS_BULK, OPS_TAIL, OPS_FULL = 28, 64, 157
REPEATS = 5                    # timed windows of the headline; the median is reported


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed steps of the measured field before each timed window (the "
                         "clocks are first warmed for about a second on the same context)")
    ap.add_argument("--repeats", type=int, default=REPEATS,
                    help="timed windows of the headline (field re-initialised each time); median")
    ap.add_argument("--fp64-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--only", default="",
                    help="run only this leg: f32 | f64 | batch | grains | temporal | musweep | walls | fig1 | fig8 | "
                         "models | cube | friction | grainruns")
    ap.add_argument("--side-steps", type=int, default=200,
                    help="timed steps of the batched and 512^3 legs")
    ap.add_argument("--coupling", default="local", choices=("local", "global", "cf"),
                    help="coupling of the timed legs (the headline is local, TI_n)")
    ap.add_argument("--no-traffic", action="store_true",
                    help="skip the two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) that measure "
                         "the headline kernel's HBM bytes per launch")
    ap.add_argument("--copy-ref", action="store_true",
                    help="first run a plain copy of 2^26 floats (256 MiB read + 256 MiB written), "
                         "the reference that scales hardware byte counters")
    ap.add_argument("--tile", type=int, nargs=2, default=None, metavar=("TX", "TY"),
                    help="tile column of the headline's tiled kernel (default: tuned at the first step)")
    ap.add_argument("--zchunk", type=int, default=0,
                    help="leading z-chunk of the headline's tiled kernel (default: tuned at the first step)")
    ap.add_argument("--traffic-child", action="store_true",
                    help="internal: the headline kernel alone, once, for a counter pass")
    return ap.parse_args()


def copy_reference(torch):
    n = 1 << 26
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    return {"elements": n, "bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}


def volume_radius(v, lam):
    """The radius R whose ideal-profile sphere holds phase volume v:
    (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16) = v, by Newton's method."""
    import math
    k = math.pi ** 2 * lam ** 2 / 16.0
    r = (3.0 * v / (4.0 * math.pi)) ** (1.0 / 3.0)
    for _ in range(50):
        r -= (r ** 3 + k * r - 3.0 * v / (4.0 * math.pi)) / (3.0 * r * r + k)
    return r


def grain_shape(d, lam):
    """Size and isotropy of the shrinking grain after the timed steps: the
    volume-equivalent radius R_V of the ideal profile's phase volume (the
    sphere of radius R holds (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16) of phi),
    the phi = 1/2 contour statistics of Sec. 3.3 (mean, extreme radii and
    eps_eff = (R_max - R_min) / (2 R_mean)), and, when given, the same from the
    radii along the configuration's seeded rays."""
    c = d["contour"]
    r = volume_radius(d["phase_volume"], lam)
    out = {"time": d["time"], "R_V": r, "R_mean": c["R_mean"], "R_min": c["R_min"],
           "R_max": c["R_max"], "eps_eff": c["eps_eff"], "contour_points": c["points"]}
    if "rays" in d:   # the same shape along the configuration's seeded rays
        rr = d["rays"]
        out.update({"rays": int(len(rr)), "ray_R_mean": float(sum(rr) / len(rr)),
                    "ray_R_min": float(min(rr)), "ray_R_max": float(max(rr)),
                    "ray_eps": float((max(rr) - min(rr)) / (2.0 * sum(rr) / len(rr)))})
    return out


def xtail_local(lam, dx=1.0, stencil=26):
    """The FP32 step's tail threshold for TI_n: below x = phi(1-phi) = 2^-24 / m_max
    every y_k = m_k x is under one ulp of 1 (m_max = 2 cosh(4 dx sqrt(j) / lambda)
    - 2 over the stencil's shells j <= 1, 2, 3), and the step takes the closed-form
    tail branch; at or above it the full coupling."""
    import math
    import numpy as np
    nsh = {6: 1, 18: 2, 26: 3}[stencil]
    h = math.sinh(2.0 * dx * math.sqrt(nsh) / lam)
    return float(np.float32(2.0 ** -24 / (4.0 * h * h)))


def point_mix(phi, xtail):
    """Fractions of points in the step's three branches, from an FP32 field (numpy
    or torch): x = phi (1 - phi) rounded as the kernel rounds it; bulk where
    x == 0, full coupling where |x| >= xtail, the tail branch elsewhere."""
    try:
        import torch
        is_t = isinstance(phi, torch.Tensor)
    except Exception:  # pragma: no cover - torch is part of the image
        is_t = False
    if is_t:
        x = phi * (1.0 - phi)
        n = x.numel()
        bulk = int((x == 0).sum().item())
        full = int((x.abs() >= xtail).sum().item())
    else:
        import numpy as np
        p = np.asarray(phi, dtype=np.float32)
        x = p * (np.float32(1.0) - p)
        n = x.size
        bulk = int(np.count_nonzero(x == 0))
        full = int(np.count_nonzero(np.abs(x) >= np.float32(xtail)))
    return {"bulk": bulk / n, "tail": (n - bulk - full) / n, "full": full / n}


def ops_per_point(mix):
    """Algorithmic FP32 operations per point update for a branch mix."""
    return OPS_BULK * mix["bulk"] + OPS_TAIL * mix["tail"] + OPS_FULL * mix["full"]


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def host_cpu():
    """Model name and usable cores of the host, from /proc/cpuinfo and the
    process's CPU affinity."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 0
    return {"cpu_model": model, "host_cores": usable, "host_cpus_total": os.cpu_count() or 0}


def warm_clocks(torch, stream, step, reinit, chunk=200, every=10, min_s=1.0, max_s=4.0, tol=0.01):
    """Run step(chunk) repeatedly, calling reinit() every `every` chunks so that
    the work per step stays that of the timed window, until at least min_s
    seconds have passed and two consecutive chunks took the same time within tol
    (at most max_s seconds): the GPU's clocks ramp up over the first fraction of
    a second of sustained work.  Returns (seconds, steps, microseconds per step of
    the last chunk)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0, n, last = time.perf_counter(), 0, None
    while True:
        if (n // chunk) % every == 0:
            reinit()
        e0.record(stream)
        step(chunk)
        e1.record(stream)
        e1.synchronize()
        n += chunk
        ms = e0.elapsed_time(e1)
        el = time.perf_counter() - t0
        if el >= max_s or (el >= min_s and last is not None and abs(ms - last) <= tol * last):
            return el, n, ms * 1e3 / chunk
        last = ms


def headline_kernel(tile=None, zchunk=0):
    """Options of the headline step: the tiled kernel with the given tile column
    and z-chunk, or (None, 0) the autotuner's choice among the compiled shapes
    and chunk lengths, timed at the first step."""
    if tile is None and not zchunk:
        return dict(kernel="auto")
    return dict(kernel="auto" if tile is None or not zchunk else "tiled", tile=tile, zchunk=zchunk)


def headline_leg(spfm, torch, w, *, steps, warmup, repeats, coupling="local", tile=None, zchunk=0,
                 rewarm_steps=300):
    """The FP32 tiled step on the grain workload.  The clocks are first brought
    to their steady state by stepping the measured context itself, its field
    re-initialised every 2000 steps (see warm_clocks; these steps are not
    measured); then `repeats` times: `rewarm_steps` untimed steps so that the
    GPU never idles between windows, the field initialised afresh (R = 60),
    stepped `warmup` times untimed, and exactly `steps` steps timed, bracketed by
    stream synchronisation (wall clock) and by HIP events on the kernel's
    stream.  The branch mix of the step is counted on the field at both ends of
    every window."""
    stream = torch.cuda.Stream()
    xt = xtail_local(w.lam, w.dx, w.stencil)
    reps = []
    with torch.cuda.stream(stream):
        kw = dict(lam=w.lam, mu=w.mu, Gamma=w.Gamma, M=w.M, dx=w.dx, stencil=w.stencil, dtype="f32",
                  coupling=coupling, dt=w.dt, stream=stream)
        if tile is None or not zchunk:
            # the autotuner times its candidates at the first step: give it warm clocks
            with spfm.Spfm(w.shape, kernel="tiled", **kw) as scratch:
                warm_clocks(torch, stream, scratch.step, lambda: scratch.init_spheres(w.centers, w.radii),
                            min_s=0.5)
        s = spfm.Spfm(w.shape, **kw, **headline_kernel(tile, zchunk))
        init = lambda: s.init_spheres(w.centers, w.radii)
        warm = warm_clocks(torch, stream, s.step, init)
        bufs = {b.data_ptr(): b for b in s._buffers}
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for _ in range(repeats):
            s.step(rewarm_steps)
            s.init_spheres(w.centers, w.radii)
            s.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            reps.append({"wall": wall, "ev_ms": e0.elapsed_time(e1)})
        # the window's state (the same in every repeat: the run is deterministic):
        # radius and branch mix at its two ends, taken after the timed windows so
        # that no reduction or allocation idles the GPU between them
        s.init_spheres(w.centers, w.radii)
        s.step(warmup)
        d0 = s.diagnostics()
        m0 = point_mix(bufs[s.field_ptr()], xt) if coupling == "local" else None
        s.step(steps)
        d1 = s.diagnostics()
        m1 = point_mix(bufs[s.field_ptr()], xt) if coupling == "local" else None
        for r in reps:
            r.update({"R0": d0["interface_position"], "R1": d1["interface_position"], "mix": (m0, m1)})
        d = s.diagnostics()
        inf = s.info()
        d["zchunk"] = inf["zchunk"]
        d["tile"] = [inf["tile_x"], inf["tile_y"]]
        d["warm"] = {"seconds": warm[0], "steps": warm[1], "us_per_step_last": warm[2]}
        d["contour"] = s.contour_stats()
        if w.rays is not None:
            d["rays"] = s.ray_radii(w.rays, centre=d["contour"]["centre"])
        s.close()
    return reps, d


def parse_counter_csv(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter-collection CSV:
    a list of (dispatch id, kernel name, value) in dispatch order."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            did = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or len(rows))
            rows.append((did, r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    rows.sort(key=lambda t: t[0])
    return rows


def traffic_from_counters(fetch_rows, write_rows, steps, copy_bytes, kernel_tag="k_step_tiled",
                          copy_tag="MulFunctor"):
    """HBM bytes per launch of the step kernel: the mean FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) of its last `steps` dispatches, each scaled by what the
    same counter reads for the plain copy kernel of known size (copy_bytes read
    and copy_bytes written per dispatch).  None when a kernel is missing."""
    def mean_last(rows, tag, k):
        v = [x for _, name, x in rows if tag in name]
        return sum(v[-k:]) / len(v[-k:]) if v else None
    f_step, w_step = mean_last(fetch_rows, kernel_tag, steps), mean_last(write_rows, kernel_tag, steps)
    f_copy, w_copy = mean_last(fetch_rows, copy_tag, 3), mean_last(write_rows, copy_tag, 3)
    if None in (f_step, w_step, f_copy, w_copy) or f_copy <= 0 or w_copy <= 0:
        return None
    kib = copy_bytes / 1024.0
    fs, ws = kib / f_copy, kib / w_copy
    name = [n for _, n, _ in fetch_rows if kernel_tag in n][-1]
    return {"bytes": (f_step * fs + w_step * ws) * 1024.0, "fetch_kib": f_step, "write_kib": w_step,
            "fetch_scale": fs, "write_scale": ws, "kernel": name}


def measure_traffic(args):
    """Two rocprofv3 counter passes over a child run of the headline kernel (the
    same window: --warmup untimed steps, then --steps, in the tile and z-chunk of
    args), FETCH_SIZE then WRITE_SIZE, with the copy reference in the same
    process.  Returns None (with the reason on stderr) if anything fails."""
    import glob
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3")
    if prof is None:
        print("traffic: rocprofv3 not found", file=sys.stderr, flush=True)
        return None
    env = dict(os.environ, TMPDIR="/tmp")
    rows = {}
    chosen = {"tile": args.tile, "zchunk": args.zchunk}
    tmp = tempfile.mkdtemp(prefix="spfm_traffic_", dir="/tmp")
    try:
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            out = os.path.join(tmp, counter)
            cmd = [prof, "--pmc", counter, "--output-format", "csv", "-d", out, "-o", "run", "--",
                   sys.executable, os.path.abspath(__file__), "--traffic-child", "--steps", str(args.steps),
                   "--warmup", str(args.warmup), "--coupling", args.coupling]
            if chosen["tile"] is not None:
                cmd += ["--tile", str(chosen["tile"][0]), str(chosen["tile"][1])]
            if chosen["zchunk"]:
                cmd += ["--zchunk", str(chosen["zchunk"])]
            print(f"traffic: {counter} pass", file=sys.stderr, flush=True)
            r = subprocess.run(cmd, cwd="/tmp", env=env, capture_output=True, text=True, timeout=240)
            # the first pass tunes the kernel; later passes and the timed run reuse its choice
            for line in reversed(r.stdout.splitlines()):
                if line.startswith("{") and "zchunk" in line:
                    c = json.loads(line)
                    chosen = {"tile": c["tile"], "zchunk": c["zchunk"]}
                    break
            files = glob.glob(os.path.join(out, "**", "*counter_collection.csv"), recursive=True)
            if r.returncode != 0 and not files:
                print(f"traffic: {counter} pass failed (rc {r.returncode}): {r.stderr[-400:]}",
                      file=sys.stderr, flush=True)
                return None
            if not files:
                print(f"traffic: no counter file for {counter}", file=sys.stderr, flush=True)
                return None
            rows[counter] = parse_counter_csv(files[0], counter)
    except (subprocess.TimeoutExpired, OSError, ValueError, KeyError) as e:
        print(f"traffic: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
        return None
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    t = traffic_from_counters(rows["FETCH_SIZE"], rows["WRITE_SIZE"], args.steps, 4 * (1 << 26))
    if t is not None:
        t.update(chosen)
    return t


def traffic_child(args):
    """One window of the headline kernel and the copy reference, for a counter pass."""
    import torch

    from paper_1910_05180_amd import inputs, spfm
    spfm.load()
    w = inputs.sphere256(mu=0.0)
    copy_reference(torch)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = spfm.Spfm(w.shape, lam=w.lam, mu=w.mu, Gamma=w.Gamma, M=w.M, dx=w.dx, stencil=w.stencil,
                      dtype="f32", coupling=args.coupling, dt=w.dt, stream=stream,
                      **headline_kernel(args.tile, args.zchunk))
        s.init_spheres(w.centers, w.radii)
        s.step(args.warmup)
        s.step(args.steps)
        torch.cuda.synchronize()
        inf = s.info()
        s.close()
    print(json.dumps({"tile": [inf["tile_x"], inf["tile_y"]], "zchunk": inf["zchunk"]}), flush=True)


def timed_run(spfm, torch, shape, w, *, dtype, kernel, steps, warmup, coupling="local", zchunk=0,
              tsteps=0, contour=False, rays=None):
    """Steps `steps` times after `warmup` untimed steps on a dedicated stream.
    Returns (wall seconds, event milliseconds) of the timed region and the
    diagnostics after it (with contour: the phi = 1/2 contour statistics)."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = spfm.Spfm(shape, lam=w.lam, mu=w.mu, Gamma=w.Gamma, M=w.M, dx=w.dx,
                      stencil=w.stencil, dtype=dtype, coupling=coupling, kernel=kernel, dt=w.dt,
                      zchunk=zchunk, tsteps=tsteps)
        s.init_spheres(w.centers, w.radii)
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms = e0.elapsed_time(e1)
        d = s.diagnostics()
        inf = s.info()
        d["zchunk"] = inf["zchunk"]
        d["tile"] = [inf["tile_x"], inf["tile_y"]]
        if contour:
            d["contour"] = s.contour_stats()
            if rays is not None:
                d["rays"] = s.ray_radii(rays, centre=d["contour"]["centre"])
        s.close()
    return wall, ev_ms, d


def batch_leg(spfm, torch, inputs, steps, warmup):
    """FP32 TI_n 26-neighbour stepping of the 64 uneven periodic slabs, one launch
    per step for all grids, captured in HIP graphs; the z-chunk is timed at the
    first (warm-up) step."""
    ws = inputs.batch64()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = spfm.SpfmBatch([w.shape for w in ws], lam=[w.lam for w in ws], mu=[w.mu for w in ws],
                           stencil=26, coupling="local")
        b.init_planar([w.hkl for w in ws], [w.offset for w in ws])
        b.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = b.points
        inf = b.info()
        b.close()
    return {"value": n * steps / wall / 1e9, "unit": "GLUPS", "grids": len(ws), "points": n,
            "steps": steps, "kernel": "tiled", "tile": [inf["tile_x"], inf["tile_y"]],
            "zchunk": inf["zchunk"], "ms_per_step": wall * 1e3 / steps,
            "kernel_ms_per_step": e0.elapsed_time(e1) / steps,
            "pct_hbm_peak": 100.0 * ALG_BYTES_F32 * n / (e0.elapsed_time(e1) / steps * 1e-3) / 1e9
            / HBM_PEAK_GBS}


def grains_leg(spfm, torch, inputs, steps, warmup, tsteps=0, coupling="local"):
    """FP32 26-neighbour step (TI_n unless coupling says otherwise) on the 512^3
    box with 300 grains (1 GiB ping-pong, far beyond the last-level cache); with
    tsteps > 1 the temporally blocked kernel fuses that many steps per pass over
    the field (z-chunk 64, the library's size rule for fused steps)."""
    w = inputs.grains512()
    steps -= steps % max(tsteps, 1)
    # one step per pass: tile and z-chunk tuned at the first (warm-up) step
    kernel, zc = ("tiled", 64) if tsteps > 1 else ("auto", 0)
    wall, ev_ms, d = timed_run(spfm, torch, w.shape, w, dtype="f32", kernel=kernel, steps=steps,
                               warmup=warmup, zchunk=zc, tsteps=tsteps, coupling=coupling)
    n = w.shape[0] * w.shape[1] * w.shape[2]
    bytes_per_point = ALG_BYTES_F32 / max(tsteps, 1)
    return {"value": n * steps / wall / 1e9, "unit": "GLUPS", "points": n, "grains": len(w.radii),
            "coupling": coupling, "steps": steps, "tsteps": max(tsteps, 1), "zchunk": d["zchunk"],
            "tile": d["tile"],
            "ms_per_step": wall * 1e3 / steps, "kernel_ms_per_step": ev_ms / steps,
            "pct_hbm_peak": 100.0 * bytes_per_point * n / (ev_ms / steps * 1e-3) / 1e9
            / HBM_PEAK_GBS}


def mu_sweep_leg(spfm, torch, inputs, warm=20, steps=120, f64_every=3):
    """The 128^3 (1,2,3) slab at lambda = 5 dx under 16 driving forces evenly
    spaced in [-0.1, 0.1] (TI_n, 26 neighbours, dt = 0.1): all 16 as one FP32
    batch (one launch per step), then every f64_every-th driving force alone
    on the FP64 tiled path.  Reports the FP32 and FP64 step rates, the
    velocity against v = -M mu / Gamma (Sec. 2.1: frictionless, no pinning
    threshold), the fitted slope and intercept of v(mu), and the FP32-FP64
    velocity difference.  The slab is 17.1 cells thick, so at |mu| = 0.1 its
    two fronts meet after about 855 steps and feel each other's tails well
    before: velocities and rates are taken over 120 steps (at most 1.2 cells
    of travel per front)."""
    import numpy as np
    sweep = inputs.planar128_mu_sweep()
    n = sweep[0].shape[0] * sweep[0].shape[1] * sweep[0].shape[2]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = spfm.SpfmBatch([w.shape for w in sweep], lam=[w.lam for w in sweep],
                           mu=[w.mu for w in sweep], stencil=26, coupling="local", dt=sweep[0].dt,
                           stream=stream)
        b.init_planar([w.hkl for w in sweep], [w.offset for w in sweep])
        b.step(warm)
        b.diagnostics()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        d32 = b.diagnostics()
        ms32 = e0.elapsed_time(e1)
        b.close()
    v32 = np.array([d["velocity"] for d in d32])
    mu = np.array([w.mu for w in sweep])
    slope, icpt = np.polyfit(mu, v32, 1)
    v64, ms64 = {}, 0.0
    for i in range(0, len(sweep), f64_every):
        w = sweep[i]
        with torch.cuda.stream(stream):
            s = spfm.Spfm(w.shape, lam=w.lam, mu=w.mu, stencil=26, coupling="local", dtype="f64",
                          kernel="tiled", dt=w.dt, stream=stream)
            s.init_planar(w.hkl, w.offset)
            s.step(warm)
            s.diagnostics()
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            v64[i] = s.diagnostics()["velocity"]
            ms64 += e0.elapsed_time(e1)
            s.close()
    rel64 = max(abs(v32[i] - v) / abs(v) for i, v in v64.items())
    return {"value": n * len(sweep) * steps / (ms32 * 1e-3) / 1e9, "unit": "GLUPS",
            "grid": "128^3, (1,2,3) slab, lambda = 5", "driving_forces": len(sweep),
            "grids_per_launch": len(sweep), "steps": steps, "ms_per_step": ms32 / steps,
            "fp64_tiled_glups": n * len(v64) * steps / (ms64 * 1e-3) / 1e9,
            "max_rel_velocity_error": float(np.max(np.abs(v32 / (-mu) - 1.0))),
            "fit_slope": float(slope), "fit_intercept": float(icpt),
            "max_rel_fp32_fp64_velocity": float(rel64)}


def walls_leg(spfm, torch, warm=400, steps=1600, coupling="local", mu0=0.05):
    """The orientation study of the paper's Sec. 3.2 on its 120 x 10 x 10 grid:
    planar fronts rotated about [001] (0, 15, 30, 45 degrees) and [011] (15, 30,
    45 degrees) between contact-angle walls (Eq. 7) that hold their
    orientation, 26 neighbours, lambda = 4 dx, mu = mu0 cos(theta), dt = 0.05,
    FP32, all seven in one walled batch (kernel AUTO: the tiled kernel, whole
    grids or x segments of the resident kernel, timed at the first step; the
    kernels compute the wall ghosts themselves), TI_n unless coupling says
    otherwise.  Reports the aggregate step rate, the relative error of each
    front's x-velocity against -M mu0 / Gamma, and the kinetic anisotropy (the
    spread of those errors over the orientations)."""
    import math
    import numpy as np
    shape, dt = (10, 10, 120), 0.05
    runs = [("001", d) for d in (0, 15, 30, 45)] + [("011", d) for d in (15, 30, 45)]
    ns = []
    for axis, deg in runs:
        th = math.radians(deg)
        ns.append((math.cos(th), math.sin(th), 0.0) if axis == "001" else
                  (math.cos(th), math.sin(th) / math.sqrt(2.0), math.sin(th) / math.sqrt(2.0)))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = spfm.SpfmBatch([shape] * len(ns), lam=4.0, mu=[mu0 * n[0] for n in ns], stencil=26,
                           coupling=coupling, dt=dt, walls=7,
                           wall_sin=[spfm.front_wall_sin(n) for n in ns], stream=stream)
        b.init_front(ns, [20.0] * len(ns))
        b.step(warm)
        d0 = b.diagnostics()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        d1 = b.diagnostics()
        ms = e0.elapsed_time(e1)
        info = b.info()
        b.close()
    worst, errs = 0.0, {}
    for (axis, deg), n, a, z in zip(runs, ns, d0, d1):
        vx = (z["interface_position"] - a["interface_position"]) / (z["time"] - a["time"]) / n[0]
        err = vx / (-mu0) - 1.0
        errs[f"{axis}:{deg}"] = err
        worst = max(worst, abs(err))
    pts = shape[0] * shape[1] * shape[2]
    return {"value": pts * steps * len(runs) / (ms * 1e-3) / 1e9, "unit": "GLUPS",
            "grid": "120x10x10 + ghost layers", "orientations": len(runs), "grids_per_launch": len(runs),
            "coupling": coupling, "mu0": mu0, "steps": steps, "us_per_step": ms * 1e3 / steps,
            "kernel": kernel_choice(spfm, info),
            "max_rel_velocity_error": worst,
            "kinetic_anisotropy": max(errs.values()) - min(errs.values()),
            "rel_velocity_error": errs}


def front_crossings(field):
    """x (in grid points) of the falling phi = 1/2 crossing of every x line of
    field (nz, ny, nx), NaN on lines without one: the one place where phi
    drops from >= 1/2 at x to < 1/2 at x + 1 (the line read periodically, so
    a periodic slab's trailing front counts and a walled front with phase 1 at
    low x is found as such), located at the zero of psi = ln((1 - phi)/phi)
    interpolated linearly between those two points.  psi is linear across the
    ideal profile of Eq. 3 (the contour reading of Eq. 8-9 at l = 1/2), so the
    crossing is exact for it at any lambda/dx.  The phase volume is not: for
    sharp profiles its change per cell of travel oscillates with the front's
    offset from the grid (about 9% of the velocity at lambda = dx), so a
    velocity taken from it over a fraction of a cell errs."""
    import numpy as np
    f = np.asarray(field, dtype=np.float64).reshape(-1, np.shape(field)[-1])
    g = np.roll(f, -1, axis=1)
    fall = (f >= 0.5) & (g < 0.5)
    ok = fall.any(axis=1)
    i = np.argmax(fall, axis=1)
    rows = np.arange(f.shape[0])
    a = np.clip(f[rows, i], 1e-300, 1.0 - 1e-16)
    b = np.clip(g[rows, i], 1e-300, 1.0 - 1e-16)
    pa, pb = np.log((1.0 - a) / a), np.log((1.0 - b) / b)
    return np.where(ok, i + pa / (pa - pb), np.nan)


def front_x(field):
    """Mean x of the front's crossings (front_crossings) over the x lines."""
    import numpy as np
    c = front_crossings(field)
    return float(np.nanmean(c)) if np.isfinite(c).any() else float("nan")


def front_shift(c0, c1, nx):
    """Mean displacement along a periodic x axis of nx points between two sets
    of per-line crossings (front_crossings), each line's difference taken
    modulo nx into [-nx/2, nx/2): an inclined front crosses every x on some
    line, so the mean of the positions themselves does not move with it."""
    import numpy as np
    d = np.asarray(c1) - np.asarray(c0)
    return float(np.nanmean((d + nx / 2.0) % nx - nx / 2.0))


def fig1_leg(spfm, torch, mu=0.1, warm_cells=2.0, cells=3.0, per_cell=10):
    """The paper's Fig. 1: a [100] slab driven at mu~ = 0.1 in a periodic box of
    120 points along x (3 x 3 cross-section, 6 neighbours, FP32): CF + h3
    at lambda~ = 4, 3, 2.5 and 2 against TI_n + h3 at lambda~ = 0.5, dt half the
    stability bound (at most 0.05).  After warm_cells of travel at -M mu /
    Gamma the trailing front is sampled per_cell times per cell of that travel
    for `cells` cells: its position front_x and the interface energy F_int of
    Eq. 1 (both fronts).  Reports the mean relative velocity error, the amplitude (half the
    range) of the velocity between samples relative to M mu / Gamma, and that
    of F_int relative to its mean."""
    import math
    import numpy as np
    shape, n = (3, 3, 120), (1.0, 0.0, 0.0)
    out = {}
    for name, coupling, lam in (("CF_lam4", "cf", 4.0), ("CF_lam3", "cf", 3.0), ("CF_lam2.5", "cf", 2.5),
                                ("CF_lam2", "cf", 2.0), ("TI_n_lam0.5", "local", 0.5)):
        bound = spfm.stable_dt(6, coupling, n, None, lam, 1.0, 1.0, mu, 1.0)
        per = int(math.ceil((1.0 / per_cell) / mu / min(0.05, 0.5 * bound)))
        dt = (1.0 / per_cell) / mu / per           # per steps = 1/per_cell cell of travel
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = spfm.Spfm(shape, lam=lam, mu=mu, stencil=6, coupling=coupling, dt=dt, stream=stream)
            s.init_planar((1, 0, 0), 0.37)
            s.step(int(round(warm_cells * per_cell)) * per)
            xs, fs = [], []
            for _ in range(int(round(cells * per_cell)) + 1):
                xs.append(front_x(s.get_field()))
                fs.append(s.energy())
                s.step(per)
            s.close()
        xs, fs = np.array(xs), np.array(fs)
        v = np.diff(xs) / (per * dt) / -mu
        out[name] = {"lam": lam, "dt": dt,
                     "mean_rel_velocity_error": float((xs[-1] - xs[0]) / (per * dt * (len(xs) - 1)) / -mu - 1.0),
                     "velocity_oscillation": float(0.5 * np.ptp(v)),
                     "energy_oscillation": float(0.5 * np.ptp(fs) / abs(fs.mean()))}
    return out


def fig8_leg(spfm, torch, plan=((4.0, 1.0, 5.0), (1.0, 1.0, 5.0), (0.5, 0.5, 2.5)), mu0=0.1):
    """The orientation study of the paper's Fig. 8 (Sec. 3.2): the seven planar
    fronts of the walls leg (rotations about [001] and [011], walls of Eq. 7 on
    all faces, 120 x 10 x 10, 26 neighbours, mu = mu0 cos(theta), FP32) at
    lambda/dx = 4, 1 and 0.5 for TI_n, three TI_<hkl> models (<100>, <110>,
    <111>) and CF, one walled batch per model and resolution.  dt is half the
    explicit stability bound (at most 0.05; at lambda = 0.5 TI_n needs about the
    paper's 1e-5).  plan holds (lambda/dx, warm-up, window): an unpinned front
    travels `warm-up` cells along x untimed, then `window` cells (the paper runs
    at least five; 2.5 at lambda = 0.5, where the steps are many).  The
    velocity is the change of front_x over the window; the relative error is
    against -M mu0 / Gamma, the x-velocity every orientation shares.  Then
    TI_n at lambda = 0.5 in FP64, one walled context per orientation, and the
    45-degree front of TI_n, TI_<100> and TI_<110> at lambda = 1 as a periodic
    slab without walls."""
    import math
    shape = (10, 10, 120)
    runs = [("001", d) for d in (0, 15, 30, 45)] + [("011", d) for d in (15, 30, 45)]
    ns = []
    for axis, deg in runs:
        th = math.radians(deg)
        ns.append((math.cos(th), math.sin(th), 0.0) if axis == "001" else
                  (math.cos(th), math.sin(th) / math.sqrt(2.0), math.sin(th) / math.sqrt(2.0)))
    models = [("TI_n", "local", (1.0, 0.0, 0.0)), ("TI_100", "global", (1.0, 0.0, 0.0)),
              ("TI_110", "global", (1.0, 1.0, 0.0)), ("TI_111", "global", (1.0, 1.0, 1.0)),
              ("CF", "cf", (1.0, 0.0, 0.0))]
    out, steps_total, ms_total = {}, 0, 0.0
    for lam, warm_cells, window in plan:
        for name, coupling, u in models:
            bound = min(spfm.stable_dt(26, coupling, u, None, lam, 1.0, 1.0, mu0 * n[0], 1.0) for n in ns)
            dt = min(0.05, 0.5 * bound)
            steps = int(math.ceil(window / mu0 / dt))
            warm = int(math.ceil(warm_cells / mu0 / dt))
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                b = spfm.SpfmBatch([shape] * len(ns), lam=lam, mu=[mu0 * n[0] for n in ns], stencil=26,
                                   coupling=coupling, u=u, dt=dt, walls=7,
                                   wall_sin=[spfm.front_wall_sin(n) for n in ns], stream=stream)
                b.init_front(ns, [20.0] * len(ns))
                b.step(warm)
                x0 = [front_x(b.get_field(i)) for i in range(len(ns))]
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                b.step(steps)
                e1.record(stream)
                stream.synchronize()
                x1 = [front_x(b.get_field(i)) for i in range(len(ns))]
                info = b.info()
                b.close()
            ms_total += e0.elapsed_time(e1)
            steps_total += steps
            errs = {f"{axis}:{deg}": (c - a) / (steps * dt) / (-mu0) - 1.0
                    for (axis, deg), a, c in zip(runs, x0, x1)}
            vals = list(errs.values())
            out[f"lam{lam:g}_{name}"] = {
                "dt": dt, "steps": steps, "kernel": kernel_choice(spfm, info),
                "rel_velocity_error": errs,
                "mean_rel_error": sum(vals) / len(vals),
                "kinetic_anisotropy": max(vals) - min(vals),
                "pinned": [k for k, v in errs.items() if v < -0.99]}
    # TI_n at lambda = 0.5 in FP64 (the FP32 fronts are limited there by the
    # storage of phi near 1): seven walled contexts, 0.05 + 0.2 cells of travel
    lam, f64 = 0.5, {}
    for (axis, deg), n in zip(runs, ns):
        dt = 0.5 * spfm.stable_dt(26, "local", n, None, lam, 1.0, 1.0, mu0 * n[0], 1.0)
        warm, steps = int(math.ceil(0.05 / mu0 / dt)), int(math.ceil(0.2 / mu0 / dt))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = spfm.Spfm(shape, lam=lam, mu=mu0 * n[0], stencil=26, dtype="f64", coupling="local", dt=dt,
                          walls=7, wall_sin=spfm.front_wall_sin(n), stream=stream)
            s.init_front(n, 20.0)
            s.step(warm)
            x0 = front_x(s.get_field())
            s.step(steps)
            x1 = front_x(s.get_field())
            s.close()
        f64[f"{axis}:{deg}"] = (x1 - x0) / (steps * dt) / (-mu0) - 1.0
    out["lam0.5_TI_n_fp64"] = {"rel_velocity_error": f64, "window_cells": 0.2,
                               "kinetic_anisotropy": max(f64.values()) - min(f64.values())}
    # the 45-degree front without walls: a periodic (1,1,0) slab in a 128 x 128 x 3
    # box at lambda = 1, 1 + 5 cells of travel, per-line displacements unwrapped
    lam, per = 1.0, {}
    n45 = (math.sqrt(0.5), math.sqrt(0.5), 0.0)
    for name, coupling, u in models[:3]:
        dt = 0.5 * spfm.stable_dt(26, coupling, u, None, lam, 1.0, 1.0, mu0 * n45[0], 1.0)
        warm, steps = int(math.ceil(1.0 / mu0 / dt)), int(math.ceil(5.0 / mu0 / dt))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = spfm.Spfm((3, 128, 128), lam=lam, mu=mu0 * n45[0], stencil=26, coupling=coupling, u=u, dt=dt,
                          stream=stream)
            s.init_planar((1, 1, 0), 0.37)
            s.step(warm)
            c0 = front_crossings(s.get_field())
            s.step(steps)
            c1 = front_crossings(s.get_field())
            s.close()
        per[name] = front_shift(c0, c1, 128) / (steps * dt) / (-mu0) - 1.0
    out["lam1_periodic_110"] = {"rel_velocity_error": per, "window_cells": 5.0}
    out["steps"] = steps_total
    out["gpu_s"] = ms_total * 1e-3
    return out


def kernel_choice(spfm, info):
    """What a batch runs, from its info: "tiled 16x8 z4", "resident whole" or
    "resident segments 8 halo 4"."""
    if info["kernel"] == spfm.KERNEL_TILED:
        return f"tiled {info['tile_x']}x{info['tile_y']} z{info['zchunk']}"
    if info["segment"]:
        return f"resident segments {info['segment']} halo {info['halo']}"
    return "resident whole"


def models_leg(spfm, torch, warm=2000, steps=4000):
    """The 1D model comparison of the paper's Fig. 7 as batched [100] slabs
    (3 x 3 x 256 periodic, two interfaces 128 dx apart, 6 neighbours, dt = 0.05,
    FP32): for each model one batch steps the slabs of every lambda~ in
    {4, 3, 2.5} and mu~ in {0.005, 0.01, 0.02, 0.05} (kernel AUTO, as above).  Reports the
    relative error of the mean interface velocity against -M mu / Gamma; then
    TI_n, TI_<100> and CF with h3 at lambda~ = 1 and 0.5 (dt at most half the
    stability bound)."""
    import math
    models = [("CF+h3", "cf", "h3"), ("CF+h5", "cf", "h5"), ("CF+h_Abel", "cf", "habel"),
              ("TI_100+h3", "global", "h3"), ("TI_n+h3", "local", "h3")]
    cases = [(lam, mu) for lam in (4.0, 3.0, 2.5) for mu in (0.005, 0.01, 0.02, 0.05)]
    shape, out, total_ms, kernels = (3, 3, 256), {}, 0.0, {}
    for name, coupling, interp in models:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            b = spfm.SpfmBatch([shape] * len(cases), lam=[c[0] for c in cases],
                               mu=[c[1] for c in cases], stencil=6, coupling=coupling,
                               interp=interp, dt=0.05, stream=stream)
            b.init_planar([(1, 0, 0)] * len(cases), [0.37] * len(cases))
            b.step(warm)
            d0 = b.diagnostics()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.step(steps)
            e1.record(stream)
            d1 = b.diagnostics()
            total_ms += e0.elapsed_time(e1)
            kernels[name] = kernel_choice(spfm, b.info())
            b.close()
        errs = {}
        for (lam, mu), a, e in zip(cases, d0, d1):
            v = (e["interface_position"] - a["interface_position"]) / (e["time"] - a["time"])
            errs[f"lam{lam:g}_mu{mu:g}"] = v / -mu - 1.0
        out[name] = errs
    # Fig. 7's sharp end: lambda~ = 1 and 0.5, where dt must shrink with the
    # stability bound; the timed window stays 200 time units, a whole number of
    # cells of travel for every mu~ here (1 to 10), over which the phase
    # volume's within-cell oscillation of sharp profiles cancels.
    sharp = {}
    for lam in (1.0, 0.5):
        mus = (0.005, 0.01, 0.02, 0.05)
        for name, coupling, interp in (("TI_n+h3", "local", "h3"), ("TI_100+h3", "global", "h3"),
                                       ("CF+h3", "cf", "h3")):
            bound = min(spfm.stable_dt(6, coupling, (1.0, 0.0, 0.0), None, lam, 1.0, 1.0, mu, 1.0)
                        for mu in mus)
            nt = int(math.ceil(200.0 / min(0.05, 0.5 * bound)))
            dt = 200.0 / nt
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                b = spfm.SpfmBatch([shape] * len(mus), lam=lam, mu=list(mus), stencil=6, coupling=coupling,
                                   interp=interp, dt=dt, stream=stream)
                b.init_planar([(1, 0, 0)] * len(mus), [0.37] * len(mus))
                b.step(nt // 2)
                d0 = b.diagnostics()
                b.step(nt)
                d1 = b.diagnostics()
                b.close()
            for mu, a, e in zip(mus, d0, d1):
                v = (e["interface_position"] - a["interface_position"]) / (e["time"] - a["time"])
                sharp.setdefault(name, {})[f"lam{lam:g}_mu{mu:g}"] = v / -mu - 1.0
            sharp.setdefault("dt", {})[f"lam{lam:g}_{name}"] = dt
    pts = shape[0] * shape[1] * shape[2] * len(cases)
    return {"value": pts * steps * len(models) / (total_ms * 1e-3) / 1e9, "unit": "GLUPS",
            "grids_per_launch": len(cases), "steps": steps,
            "us_per_step": total_ms * 1e3 / (steps * len(models)), "kernel": kernels,
            "rel_velocity_error": out, "sharp_rel_velocity_error": sharp}


def cube_leg(spfm, torch, steps=3000, sweep=((4.0, 2.0, 1.5, 1.2, 1.0), 300.0)):
    """The residual-anisotropy study of the paper's Fig. 9 on its 60^3 grid: a
    cube particle (edge 30 dx) relaxed at constant volume (mu chosen on the
    device at every step), FP32, 26 neighbours.  Timed: TI_n at lambda~ = 4
    and 2 and CF at lambda~ = 2 (dt = 0.1, `steps` steps); reports eps_eff of
    the phi = 1/2 contour and the step rate.  Then Fig. 9b: eps_eff after
    sweep[1] time units for TI_n, TI_<100> (aligned with the cube's faces),
    TI_<110>, TI_<120> and CF at each lambda~ of sweep[0], dt half the
    explicit bound (at most 0.1)."""
    import math
    n, edge = 60, 30.0
    lo = (n - edge) / 2 + 0.25
    out, total_ms = {}, 0.0

    def relax(lam, coupling, u, dt, nsteps, timed):
        nonlocal total_ms
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = spfm.Spfm((n, n, n), lam=lam, mu=-0.1, stencil=26, coupling=coupling, u=u, dt=dt,
                          conserve_volume=True, stream=stream)
            s.init_box((lo, lo, lo), (lo + edge, lo + edge, lo + edge))
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(nsteps)
            e1.record(stream)
            c = s.contour_stats()
            d = s.diagnostics()
            if timed:
                total_ms += e0.elapsed_time(e1)
            s.close()
        return {"eps_eff": c["eps_eff"], "R_mean": c["R_mean"], "mu": d["mu"]}

    for name, lam, coupling in (("TI_n_lam4", 4.0, "local"), ("TI_n_lam2", 2.0, "local"),
                                ("CF_lam2", 2.0, "cf")):
        out[name] = relax(lam, coupling, (1.0, 0.0, 0.0), 0.1, steps, True)
    pts = n ** 3
    res = {"value": pts * steps * 3 / (total_ms * 1e-3) / 1e9, "unit": "GLUPS", "grid": "60^3",
           "steps": steps, "us_per_step": total_ms * 1e3 / (3 * steps), "runs": out}
    if sweep:
        lams, T = sweep
        models = [("TI_n", "local", (1.0, 0.0, 0.0)), ("TI_100", "global", (1.0, 0.0, 0.0)),
                  ("TI_110", "global", (1.0, 1.0, 0.0)), ("TI_120", "global", (1.0, 2.0, 0.0)),
                  ("CF", "cf", (1.0, 0.0, 0.0))]
        table = {}
        for lam in lams:
            for name, coupling, u in models:
                dt = min(0.1, 0.5 * spfm.stable_dt(26, coupling, u, None, lam, 1.0, 1.0, 0.2, 1.0))
                r = relax(lam, coupling, u, dt, int(math.ceil(T / dt)), False)
                table[f"lam{lam:g}_{name}"] = {"eps_eff": r["eps_eff"], "dt": dt}
        res["fig9b_eps_eff"] = table
        res["fig9b_time"] = T
    return res


def sphere_law(r0, mu, t, M, Gamma, sigma, n=2000):
    """R(t) of a sphere under the sharp-interface law dR/dt = -(M / Gamma)
    (mu + 2 sigma / R) (Sec. 3.3: planar velocity -M mu / Gamma along the outward
    normal of the phi = 1 grain, curvature 2 / R), by RK4 in n steps."""
    f = lambda r: -(M / Gamma) * (mu + 2.0 * sigma / r)
    r, h = r0, t / n
    for _ in range(n):
        k1 = f(r)
        k2 = f(r + 0.5 * h * k1)
        k3 = f(r + 0.5 * h * k2)
        k4 = f(r + h * k3)
        r += h * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
    return r


def grain_runs_leg(spfm, torch, inputs, steps=5000, every=500, mus=(0.0, 0.02)):
    """The 256^3 grain (R0 = 60, lambda = 4, FP32, TI_n, 26 neighbours) run for
    its full 5000 steps at mu = 0 and mu = 0.02: the volume-equivalent radius
    R_V(t) every `every` steps against the sharp-interface law (at mu = 0, R^2
    falls at 4 M sigma / Gamma with sigma = 2 Gamma / (3 C_Gamma)), and the shape
    at the end (contour eps_eff, radii along the 1000 seeded rays)."""
    w0 = inputs.sphere256(mu=0.0)
    out = {}
    for mu in mus:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = spfm.Spfm(w0.shape, lam=w0.lam, mu=mu, Gamma=w0.Gamma, M=w0.M, dx=w0.dx,
                          stencil=w0.stencil, dtype="f32", coupling="local", dt=w0.dt, stream=stream)
            s.init_spheres(w0.centers, w0.radii)
            inf = s.info()
            sigma = 2.0 * inf["Gamma"] / (3.0 * inf["C_Gamma"])
            pts, worst = [], 0.0
            for i in range(steps // every + 1):
                if i:
                    s.step(every)
                d = s.diagnostics()
                r = volume_radius(d["phase_volume"], w0.lam)
                law = sphere_law(w0.radii[0], mu, d["time"], inf["M"], inf["Gamma"], sigma)
                pts.append([d["time"], r, law])
                worst = max(worst, abs(r - law) / max(abs(w0.radii[0] - law), 1e-9)) if i else worst
            d = s.diagnostics()
            d["contour"] = s.contour_stats()
            d["rays"] = s.ray_radii(w0.rays, centre=d["contour"]["centre"])
            shape = grain_shape(d, w0.lam)
            s.close()
        out[f"mu{mu:g}"] = {"steps": steps, "R_V_vs_law": pts,
                            "max_rel_dev_of_change": worst, "lam_over_R_end": w0.lam / pts[-1][1],
                            "eps_eff": shape["eps_eff"], "ray_eps": shape.get("ray_eps")}
    return out


def friction_leg(spfm):
    """The grid friction force study of the paper's Fig. 3: oscillation
    amplitude of the total force on an ideal front moved through the grid (12
    positions over one grid spacing) in the 300 x 1 x 1 system, for CF,
    TI_<120> and TI_n at lambda~ = 1 and 3, orientations about [001] and [011]
    from 0 to 75 degrees every 15 (FP64, 26 neighbours, one step per position).
    The line crosses the front once; as n_x -> 0 the line sum (which counts
    1/n_x of the front per unit area) diverges, so 90 degrees is left out."""
    import math
    import time

    from paper_1910_05180_amd import friction
    u120 = (1 / math.sqrt(5), 2 / math.sqrt(5), 0.0)
    models = (("CF", "cf", (1.0, 0.0, 0.0)), ("TI_120", "global", u120), ("TI_n", "local", (1.0, 0.0, 0.0)))
    out, t0 = {}, time.perf_counter()
    for lam in (1.0, 3.0):
        for name, coupling, u in models:
            row = {}
            for axis in ("001", "011"):
                for deg in range(0, 76, 15):
                    t = math.radians(deg)
                    n = (math.cos(t), math.sin(t), 0.0) if axis == "001" else \
                        (math.cos(t), math.sin(t) / math.sqrt(2), math.sin(t) / math.sqrt(2))
                    row[f"{axis}:{deg}"] = friction.amplitude(spfm, coupling=coupling, lam=lam, n=n, u=u)
            out[f"{name}_lam{lam:g}"] = row
    return {"amplitude": out, "wall_s": time.perf_counter() - t0,
            "system": "300x1x1 between exact contact-angle walls, FP64"}


def cpu_baseline(w, steps):
    import numpy as np

    import oracle
    shape = w.shape
    phi = oracle.init_spheres(shape, w.centers, w.radii, lam=w.lam, dx=w.dx)
    p = oracle.params(shape, lam=w.lam, mu=w.mu, Gamma=w.Gamma, M=w.M, dx=w.dx, dt=w.dt,
                      stencil=w.stencil, coupling="local", eps=1e-300)
    t0 = time.perf_counter()
    phi = oracle.step(p, phi, steps)
    dt = time.perf_counter() - t0
    n = int(np.prod(shape))
    return {"value": n * steps / dt / 1e9, "unit": "GLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", **host_cpu(),
            "sample": f"{steps} FP64 steps of the full {shape[2]}^3 grain workload "
                      f"(26 neighbours, TI_n), {dt:.1f} s wall"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.traffic_child:
        traffic_child(args)
        return
    traffic = None
    import torch

    from paper_1910_05180_amd import inputs, spfm
    spfm.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = inputs.sphere256(mu=0.0)
    npts = w.shape[0] * w.shape[1] * w.shape[2]

    out = {"metric": "GLUPS + % HBM peak, 256^3 FP32 26-nbr SPFM step vs FP64 plain"}
    if args.copy_ref:
        out["copy_reference"] = copy_reference(torch)
    f32 = f64 = None
    if args.only in ("", "f32"):
        print("leg: f32 headline", file=sys.stderr, flush=True)
        reps, d = headline_leg(spfm, torch, w, steps=args.steps, warmup=args.warmup,
                               repeats=max(1, args.repeats), coupling=args.coupling, tile=args.tile,
                               zchunk=args.zchunk)
        f32 = {"reps": reps, "diag": d}
        if not args.no_traffic:
            # two counter passes in child processes, on the configuration timed here
            print("leg: traffic counters", file=sys.stderr, flush=True)
            targs = argparse.Namespace(**vars(args))
            targs.tile, targs.zchunk = d["tile"], d["zchunk"]
            traffic = measure_traffic(targs)
    if args.only in ("", "f64"):
        print("leg: f64 plain", file=sys.stderr, flush=True)
        wall64, ev64, d64 = timed_run(spfm, torch, w.shape, w, dtype="f64", kernel="plain",
                                      steps=args.fp64_steps, warmup=min(args.warmup, 5),
                                      coupling=args.coupling)
        f64 = {"wall": wall64, "ev_ms": ev64, "diag": d64}

    if f32 is not None:
        steps, reps = args.steps, f32["reps"]
        wall = median([r["wall"] for r in reps])
        kern_ms = median([r["ev_ms"] for r in reps]) / steps     # average step-kernel duration
        glups = npts * steps / wall / 1e9
        achieved = ALG_BYTES_F32 * npts / (kern_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": traffic["bytes"] if traffic else None}
        window = {"steps": [args.warmup, args.warmup + steps],
                  "R_V": [median([r["R0"] for r in reps]), median([r["R1"] for r in reps])],
                  "repeats": len(reps), "clock_warmup": f32["diag"]["warm"],
                  "glups_each": [npts * steps / r["wall"] / 1e9 for r in reps],
                  "kernel_us_each": [r["ev_ms"] * 1e3 / steps for r in reps]}
        issue = None
        if args.coupling == "local":
            mixes = [m for r in reps for m in r["mix"]]
            mix = {k: sum(m[k] for m in mixes) / len(mixes) for k in ("bulk", "tail", "full")}
            ops = ops_per_point(mix)
            tops = ops * npts / (kern_ms * 1e-3) / 1e12
            issue = {"achieved": tops, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                     "frac": tops / VALU_PEAK_TOPS, "ops_per_point": ops, "point_mix": mix}
        out.update({
            "value": glups, "unit": "GLUPS", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "grain256: 256^3 periodic grid, one grain R=60 dx at the "
                                   "centre (ideal radial profile), lambda=4 dx, mu=0, "
                                   "Gamma=M=dx=1, dt=0.1, 26 neighbours, TI_n local normal, "
                                   "FP32 tiled kernel",
                       "points": npts, "stencil": 26, "coupling": args.coupling,
                       "kernel": "tiled", "tile": f32["diag"]["tile"], "zchunk": f32["diag"]["zchunk"]},
            "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBS,
            "hbm_achieved_gbs": achieved,
            "roofline": roofline,
            "issue_rate": issue,
            "traffic_counters": traffic,
            "window": window,
            "kernel_ms_per_step": kern_ms,
            "phi_range": [f32["diag"]["phi_min"], f32["diag"]["phi_max"]],
            "grain": grain_shape(f32["diag"], w.lam),
        })
    if f64 is not None:
        s64 = args.fp64_steps
        g64 = npts * s64 / f64["wall"] / 1e9
        k64 = f64["ev_ms"] / s64
        out["fp64_plain"] = {"value": g64, "unit": "GLUPS", "steps": s64,
                             "ms_per_step": f64["wall"] * 1e3 / s64, "kernel_ms_per_step": k64,
                             "pct_hbm_peak": 100.0 * ALG_BYTES_F64 * npts / (k64 * 1e-3) / 1e9
                             / HBM_PEAK_GBS}
        if f32 is not None:
            out["speedup_vs_fp64_plain"] = out["value"] / g64
    # The side legs: (--only name, label, [(output key, call)]).  A leg that
    # raises is recorded under leg_errors and the others still run, so the
    # headline line is printed whatever happens to them.
    legs = [
        ("batch", "batch64", [("batch64", lambda: batch_leg(spfm, torch, inputs, args.side_steps, 10))]),
        ("grains", "grains512", [("grains512", lambda: grains_leg(spfm, torch, inputs, args.side_steps, 10))]),
        ("temporal", "temporal", [
            ("grains512_temporal2", lambda: grains_leg(spfm, torch, inputs, args.side_steps, 10, tsteps=2)),
            # CF: the HBM-bound step, where fusing steps pays
            ("grains512_cf", lambda: grains_leg(spfm, torch, inputs, args.side_steps, 10, coupling="cf")),
            ("grains512_cf_temporal3", lambda: grains_leg(spfm, torch, inputs, args.side_steps, 10, tsteps=3,
                                                          coupling="cf"))]),
        ("musweep", "mu sweep", [("mu_sweep128", lambda: mu_sweep_leg(spfm, torch, inputs))]),
        ("walls", "walls", [
            ("orientation120_walls", lambda: walls_leg(spfm, torch)),
            # the continuum-field control at the paper's mu0: friction makes it orientation dependent
            ("orientation120_walls_cf", lambda: walls_leg(spfm, torch, coupling="cf", mu0=0.1))]),
        ("fig1", "fig1", [("fig1_pinning", lambda: fig1_leg(spfm, torch))]),
        ("fig8", "fig8", [("fig8_orientation", lambda: fig8_leg(spfm, torch))]),
        ("models", "models", [("fig7_models", lambda: models_leg(spfm, torch))]),
        ("cube", "cube", [("fig9_cube60", lambda: cube_leg(spfm, torch))]),
        ("friction", "friction", [("fig3_friction", lambda: friction_leg(spfm))]),
        ("grainruns", "grain runs", [("grain256_runs", lambda: grain_runs_leg(spfm, torch, inputs))]),
    ]
    for name, label, parts in legs:
        if args.only not in ("", name):
            continue
        print(f"leg: {label}", file=sys.stderr, flush=True)
        for key, call in parts:
            try:
                out[key] = call()
            except Exception as e:   # recorded, not hidden: the line carries it
                import traceback
                traceback.print_exc()
                out.setdefault("leg_errors", {})[key] = f"{type(e).__name__}: {e}"
    if not args.no_cpu and f32 is not None:
        print("leg: cpu oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
