"""Host-side pieces of bench.py: the per-kernel work table, the measured
traffic lookup (tied to the sources it was measured on) and the one-GPU
guard."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_work_rates_and_units():
    b = _bench()
    # (total ms, launches, work) over two steps
    br = {"k_gemm": (20.0, 10, 2.0e11), "k_copy": (4.0, 6, 1.6e10), "k_spmv": (1.0, 2, 0.0)}
    out = b.kernel_work(br, 2, "FP64")
    g = out["k_gemm"]
    assert g["ms"] == 10.0 and g["calls"] == 5
    assert abs(g["gflop"] - 100.0) < 1e-9
    assert abs(g["tflops"] - 10.0) < 1e-9            # 2e11 flops in 20 ms
    assert abs(g["frac_peak"] - round(10.0 / 78.6, 4)) < 1e-12
    c = out["k_copy"]
    assert abs(c["gbytes"] - 8.0) < 1e-9 and abs(c["gbs"] - 4000.0) < 1e-9
    assert abs(c["frac_hbm"] - 0.5) < 1e-12
    assert "k_spmv" not in out                         # no recorded work
    assert b.kernel_work(br, 2, "FP32")["k_gemm"]["peak_tflops"] == 157.3


def test_measured_traffic_follows_the_sources():
    b = _bench()
    assert b.measured_traffic("k_cpqr_coop", "no_such_workload") is None
    assert b.measured_traffic("k_gemm", "fv3d_128") is None
    rel = "paper_2007_00789_amd/csrc/kernels_qr_coop.hip"
    with open(os.path.join(ROOT, rel), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    b.MEASURED_TRAFFIC[("k_test", "w")] = {"sources": {rel: digest}, "fetch_kib": 10.0,
                                           "write_kib": 4.0, "fetch_scale": 2.0,
                                           "write_scale": 1.0}
    assert b.measured_traffic("k_test", "w") == 1024.0 * (10.0 * 2.0 + 4.0)
    b.MEASURED_TRAFFIC[("k_test", "w")]["sources"] = {rel: "0" * 64}   # sources changed
    assert b.measured_traffic("k_test", "w") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr
