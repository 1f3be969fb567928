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
    """VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
    second (39.3 T, a quarter of the 157.3 TFLOP/s that counts an FMA as two
    flops and packed FP32 as two lanes); HBM: 8 TB/s; 8 algorithmic bytes per
    FP32 point and step."""
    assert bench.VALU_PEAK_TOPS == pytest.approx(39.3216)
    assert bench.VALU_PEAK_TOPS * 4 == pytest.approx(157.3, rel=1e-3)
    assert bench.HBM_PEAK_GBS == 8000.0 and bench.ALG_BYTES_F32 == 8
    assert bench.ALG_OPS_LOCAL26 == pytest.approx(65.9, abs=0.05)
