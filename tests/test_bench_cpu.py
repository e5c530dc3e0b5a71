"""Host-side logic of bench.py (no GPU): the algorithmic byte counts of the
roofline, the scaling of the rocprofv3 traffic counters and its staleness
check, and the one-GPU guard."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench
import paper_1706_02740_amd as sft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_headline():
    """N = 2^22, s = 64: M = 43,648 nodes per band, Q = 16 bands, 13 taps.
    The gather reads 13 complex64 per node and writes Q samples per node; the
    short DFTs read every sample once (5.59 MB per transform).  Their full
    write of the bins is overhead: the method reads bins only at the heavy
    ones and at accepted candidates."""
    info = sft.describe(2 ** 22, 64)
    assert info["M"] == 43_648 and info["Q"] == 16
    work = bench.kernel_work(info)
    gather_bytes, gather_flops, gather_extra = work["k_gather"]
    assert gather_bytes == 43_648 * 13 * 8 + 16 * 43_648 * 8          # 4.54 MB + 5.59 MB
    assert gather_flops == 16 * 43_648 * 13 * 8 and gather_extra == 0
    dft_bytes, _, dft_extra = work["k_dft_mx"]
    assert dft_bytes == 16 * 43_648 * 8 == work["k_dft"][0] == dft_extra


def test_roofline_object_from_algorithmic_bytes():
    """frac = algorithmic bytes per launch / mean launch time / 8 TB/s: 256
    headline transforms' sample reads (1.430 GB) in 0.954 ms are 0.187 of
    the peak; the E write is reported as overhead, not counted."""
    info = sft.describe(2 ** 22, 64)
    work = bench.kernel_work(info)
    kern = {"k_dft_mx": {"launches": 20, "total_ms": 20 * 0.954, "avg_ms": 0.954}}
    roof = bench.roofline_of("k_dft_mx", work, kern, {"k_dft_mx": 256.0}, info)
    assert roof["algorithmic_bytes_per_launch"] == 256 * 16 * 43_648 * 8
    assert roof["frac"] == pytest.approx(256 * 16 * 43_648 * 8 / 0.954e-3 / 8e12)
    assert 0.18 < roof["frac"] < 0.19
    assert roof["overhead_bytes_per_launch"] == roof["algorithmic_bytes_per_launch"]


def test_matrix_core_gather_roofline_is_the_fp32_mfma_peak():
    """Theorem 4's preset at N = 2^22 (45 taps, Q = 40): the band sums are
    8 flops per tap, band and node (a complex tap times a complex phasor,
    accumulated), 0.628 GFLOP per transform; 256 transforms in 3.3 ms are
    48.7 TFLOP/s, 0.31 of the FP32 matrix-core peak (157.3 TFLOP/s)."""
    info = sft.describe(2 ** 22, 64, preset="theory")
    assert info["kappa"] == 22 and info["Q"] == 40
    work = bench.kernel_work(info)
    assert work["k_gather_mx"] == work["k_gather"]
    flops = work["k_gather_mx"][1]
    assert flops == 40 * 43_648 * 45 * 8
    kern = {"k_gather_mx": {"launches": 5, "total_ms": 5 * 3.3, "avg_ms": 3.3}}
    roof = bench.roofline_of("k_gather_mx", work, kern, {"k_gather_mx": 256.0}, info)
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s" and roof["peak"] == 157.3
    assert roof["achieved"] == pytest.approx(256 * flops / 3.3e-3 / 1e12)
    assert 0.30 < roof["frac"] < 0.32


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["usable_cpus"] <= h["nproc"]
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)


def _traffic_file(path, sha, fetch_kib, write_kib):
    with open(path, "w") as fh:
        fh.write("# test\n")
        fh.write(f"kernels_sha256: {sha}\ncopy_bytes: {2 ** 30}\ntransforms_per_launch: 256\n")
        fh.write(f"copy fetch_kib: {2 ** 20 / 2}\ncopy write_kib: {2 ** 20}\n")
        fh.write(f"k_dft_mx fetch_kib: {fetch_kib}\nk_dft_mx write_kib: {write_kib}\n")


def test_traffic_counters_are_scaled_by_the_copy_calibration(tmp_path, monkeypatch):
    """A copy of 1 GiB whose FETCH_SIZE reads half its bytes gives a fetch
    scale of 2 and a write scale of 1."""
    sha = hashlib.sha256(open(bench.KERNELS_SRC, "rb").read()).hexdigest()
    f = tmp_path / "traffic.txt"
    _traffic_file(f, sha, fetch_kib=1000.0, write_kib=3000.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    tr = bench.measured_traffic("k_dft_mx")
    assert tr["fetch_scale"] == pytest.approx(2.0) and tr["write_scale"] == pytest.approx(1.0)
    assert tr["fetch_bytes"] == pytest.approx(1000.0 * 1024 * 2)
    assert tr["bytes"] == pytest.approx(1000.0 * 1024 * 2 + 3000.0 * 1024)
    assert tr["transforms_per_launch"] == 256


def test_traffic_counters_of_other_kernel_sources_are_ignored(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    _traffic_file(f, "0" * 64, fetch_kib=1000.0, write_kib=3000.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("k_dft_mx") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("k_dft_mx") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
