"""Host-side logic of bench.py, without a GPU: the one-GPU contract, the
inversion of the ideal profile's phase volume used for the grain's radius,
and the figures the roofline is priced against."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    """The benchmark runs on one GPU; the refusal happens before torch or the
    library is loaded."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == n and "one GPU" in msg["error"]


@pytest.mark.parametrize("radius,lam", [(60.0, 4.0), (48.9776, 4.0), (7.5, 2.5), (2.0, 6.0)])
def test_grain_radius_inverts_the_ideal_phase_volume(radius, lam):
    """A sphere of the ideal radial profile holds (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16)
    of phi; grain_shape recovers R from that volume."""
    v = 4.0 * math.pi / 3.0 * (radius ** 3 + radius * math.pi ** 2 * lam ** 2 / 16.0)
    d = {"time": 1.0, "phase_volume": v,
         "contour": {"R_mean": radius, "R_min": radius, "R_max": radius, "eps_eff": 0.0, "points": 1}}
    g = bench.grain_shape(d, lam)
    assert g["R_V"] == pytest.approx(radius, rel=1e-13)


def test_roofline_peaks():
    """VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
    second (39.3 T, a quarter of the 157.3 TFLOP/s that counts an FMA as two
    flops and packed FP32 as two lanes); HBM: 8 TB/s; 8 algorithmic bytes per
    FP32 point and step."""
    assert bench.VALU_PEAK_TOPS == pytest.approx(39.3216)
    assert bench.VALU_PEAK_TOPS * 4 == pytest.approx(157.3, rel=1e-3)
    assert bench.HBM_PEAK_GBS == 8000.0 and bench.ALG_BYTES_F32 == 8
    assert bench.ops_per_point({"bulk": 0.131, "tail": 0.798, "full": 0.071}) == pytest.approx(65.9, abs=0.05)


def test_tail_threshold_and_point_mix():
    """The tail threshold 2^-24 / (2 cosh(4 sqrt(3) / lambda) - 2) for 26 neighbours,
    and the branch classes of an ideal planar profile: bulk where phi(1-phi)
    rounds to 0 in FP32, full coupling within the band where it exceeds the
    threshold, the tail elsewhere."""
    import numpy as np
    lam = 4.0
    xt = bench.xtail_local(lam)
    assert xt == pytest.approx(2.0 ** -24 / (2.0 * math.cosh(4.0 * math.sqrt(3.0) / lam) - 2.0), rel=1e-7)
    s = np.arange(-200, 200) + 0.25
    phi = (0.5 * (1.0 - np.tanh(2.0 * s / lam))).astype(np.float32)
    mix = bench.point_mix(phi, xt)
    assert sum(mix.values()) == pytest.approx(1.0)
    x = phi.astype(np.float64) * (1.0 - phi.astype(np.float64))
    # the full band: x >= xt, i.e. |s| below about (lambda/4) ln(1/xt)
    half = lam / 4.0 * math.log(1.0 / xt)
    assert mix["full"] * s.size == pytest.approx(2 * half, abs=3)
    assert mix["bulk"] > 0 and mix["tail"] > 0
    assert np.count_nonzero(x == 0) >= mix["bulk"] * s.size


def test_traffic_from_counter_rows(tmp_path):
    """Per-launch HBM bytes from the rocprofv3 counter CSV: the mean of the step
    kernel's last dispatches, each counter scaled by the copy reference's reading
    of a known size."""
    csv_text = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i in range(3):
        csv_text.append(f"{i},\"void at::native::elementwise<MulFunctor<float>>\",FETCH_SIZE,131072.0")
    for i in range(3, 8):
        csv_text.append(f"{i},\"void spfm::k_step_tiled<float, 26, 0, false>\",FETCH_SIZE,{40000.0 + i}")
    p = tmp_path / "run_counter_collection.csv"
    p.write_text("\n".join(csv_text) + "\n")
    fetch = bench.parse_counter_csv(str(p), "FETCH_SIZE")
    assert len(fetch) == 8
    write = [(i, n, 262144.0 if "Mul" in n else 65536.0) for i, n, _ in fetch]
    t = bench.traffic_from_counters(fetch, write, steps=2, copy_bytes=4 * (1 << 26))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_kib"] == pytest.approx(40006.5)
    assert t["bytes"] == pytest.approx((40006.5 * 2.0 + 65536.0) * 1024.0)
    assert bench.traffic_from_counters(fetch, [], 2, 4 * (1 << 26)) is None


def test_median():
    assert bench.median([3.0, 1.0, 2.0]) == 2.0
    assert bench.median([4.0, 1.0, 2.0, 3.0]) == 2.5


@pytest.mark.parametrize("lam", [4.0, 1.0, 0.5])
@pytest.mark.parametrize("n", [(1.0, 0.0, 0.0), (0.9, 0.3, 0.1), (0.7, 0.5, 0.5)])
def test_front_x_is_exact_for_ideal_fronts(lam, n):
    """front_x locates a planar front by the zeros of psi = ln((1 - phi)/phi)
    along x; psi is linear across the ideal profile of Eq. 3, so moving the
    front by d along n moves front_x by d / n_x exactly, at any lambda/dx."""
    import numpy as np
    import oracle
    n = np.asarray(n) / np.linalg.norm(n)
    offs = [0.0, 0.13, 0.5, 0.77, 1.6]
    xs = [bench.front_x(oracle.front((10, 10, 120), n, o, lam=lam)) for o in offs]
    assert np.allclose(np.diff(xs), np.diff(offs) / n[0], rtol=0, atol=1e-9)


def test_phase_volume_is_not_an_exact_front_position_for_sharp_profiles():
    """Why front_x: at lambda = dx the phase volume of the ideal profile is
    not linear in the front's offset (its slope varies by about 9% within a
    cell), while front_x is."""
    import numpy as np
    import oracle
    n = (1.0, 0.0, 0.0)
    offs = np.linspace(0.0, 1.0, 9)
    vol = np.array([oracle.front((2, 2, 60), n, o, lam=1.0).sum() / 4.0 for o in offs])
    slope = np.diff(vol) / np.diff(offs)
    assert np.ptp(slope) > 0.1
    xs = np.array([bench.front_x(oracle.front((2, 2, 60), n, o, lam=1.0)) for o in offs])
    assert np.allclose(np.diff(xs) / np.diff(offs), 1.0, atol=1e-9)


@pytest.mark.parametrize("lam", [4.0, 1.0])
def test_front_shift_follows_an_inclined_periodic_slab(lam):
    """On a periodic (1,1,0) slab the crossings cover every x of the box, so
    their mean stays put as the slab moves; front_shift unwraps each line's
    displacement and recovers the shift along x, d / n_x, exactly."""
    import numpy as np
    import oracle
    shape, n_x = (3, 64, 64), np.sqrt(0.5)
    c0 = bench.front_crossings(oracle.init_planar(shape, (1, 1, 0), 0.37, lam=lam))
    for d in (0.3, 1.7, 4.1):
        c1 = bench.front_crossings(oracle.init_planar(shape, (1, 1, 0), 0.37 + d, lam=lam))
        assert bench.front_shift(c0, c1, 64) == pytest.approx(d / n_x, abs=1e-9)
