"""bench.py's command-line contract that holds without a GPU: more than one
GPU is refused with a message and a non-zero status before anything runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_roofline_fields():
    """The roofline block's arithmetic: 40 integer ops per pixel-pass per
    launch over the average launch time, against the ALU peak; bytes and the
    method-work fraction beside it."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench._roofline(px_passes=10**9, alg_bytes=2 * 10**9, launches=10, kernel_ms=4.0,
                        traffic=10**8, x_method=10**8, timing="t", steps=2)
    assert r["bound"] == "alu" and r["unit"] == "Tops/s"
    assert abs(bench.ALU_PEAK_TOPS - 39.3216) < 1e-9
    # 4e10 ops over 4 ms = 10 Tops/s
    assert abs(r["achieved"] - 10.0) < 1e-9
    assert abs(r["frac"] - round(10.0 / bench.ALU_PEAK_TOPS, 4)) < 1e-12
    assert r["launches_per_step"] == 5 and abs(r["avg_launch_us"] - 400.0) < 1e-9
    # 2e9 bytes over 4 ms = 500 GB/s; traffic 1e8 B per launch over 0.4 ms
    assert abs(r["hbm"]["achieved"] - 500.0) < 1e-9
    assert abs(r["hbm"]["traffic_GBps"] - 250.0) < 1e-9
    assert abs(r["method_work_frac"] - round(1.0 / bench.ALU_PEAK_TOPS, 4)) < 1e-12
    z = bench._roofline(1, 1, 0, 0.0, None, 1, "t")
    assert z["achieved"] is None and z["frac"] is None and z["launches_per_step"] == 1
