"""Host-side checks of the benchmark script (no GPU): the one-GPU guard and the
parser that reads HBM traffic from a committed profiler summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.fixture()
def bench_module(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    return bench


def _summary(path, sha, fetch_kib, write_kib):
    path.write_text(f"# a summary\nkernel_source_sha256: {sha}\n"
                    f"fetch_kib_per_dispatch: {fetch_kib}\nwrite_kib_per_dispatch: {write_kib}\n"
                    "fetch_scale: 2.0\nwrite_scale: 1.0\n")


def test_traffic_is_read_and_scaled(bench_module, tmp_path):
    _summary(tmp_path / "profiles" / "pmc_csa_u16_2p33.txt", "abc123", 8388608, 32)
    t = bench_module.read_traffic("csa", "u16_2p33", "abc123", 1 << 34)
    assert t["fetch_bytes"] == 8388608 * 1024 * 2.0
    assert t["write_bytes"] == 32 * 1024
    assert t["hbm_bytes"] == t["fetch_bytes"] + t["write_bytes"]
    assert abs(t["vs_algorithmic"] - (t["hbm_bytes"] / 2**34)) < 1e-12


def test_traffic_of_other_kernel_source_is_not_reported(bench_module, tmp_path):
    _summary(tmp_path / "profiles" / "pmc_csa_u16_2p33.txt", "abc123", 8388608, 32)
    assert bench_module.read_traffic("csa", "u16_2p33", "def456", 1 << 34) is None
    assert bench_module.read_traffic("csa", "u8_2p34", "abc123", 1 << 34) is None


def test_kernel_source_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.kernel_source_hash()


def test_unknown_leg_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--legs", "single,nope"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "--legs takes" in r.stderr
    assert r.stdout == ""
