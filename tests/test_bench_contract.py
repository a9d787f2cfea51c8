"""Host-side checks of bench.py's output contract (no GPU): the roofline
entry's fields, bound and fraction, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("cls,bound,unit", [("ttm_matvec", "hbm", "GB/s"), ("gemm_f64", "mfma", "TFLOP/s"),
                                            ("schur_qr", "alu", "TFLOP/s")])
def test_roofline_entry_fields_bound_and_fraction(cls, bound, unit):
    st = {"ms": 2.0, "launches": 4, "bytes": 8.0e6, "flops": 4.0e9}
    r = bench.roofline_entry(cls, st, traffic=123.0)
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r
    assert r["bound"] == bound and r["unit"] == unit and r["traffic"] == 123.0
    per_launch_s = 2.0e-3 / 4
    if bound == "hbm":
        assert r["peak"] == bench.PEAK_HBM_GBS
        assert r["achieved"] == pytest.approx(8.0e6 / 4 / per_launch_s / 1e9)
    else:
        assert r["peak"] == bench.PEAK_FP64_TFLOPS
        assert r["achieved"] == pytest.approx(4.0e9 / 4 / per_launch_s / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "--gpus 2" in p.stderr and p.stdout == ""
