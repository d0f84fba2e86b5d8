"""Host logic of bench.py that needs no GPU: the one-GPU guard, the algorithmic
byte and pair counts the roofline is priced with, and the rule that measured HBM
traffic is reported only for the kernel sources it was taken on."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_particle_step():
    # half list of Fig. 1: rho (2 pi / 3) r_list^3 partners per particle, 4 bytes each,
    # plus FP64 q and v read and written (4 x 24 bytes)
    n_half = 0.5 * (2.0 * math.pi / 3.0) * 2.8 ** 3
    assert n_half == pytest.approx(22.99, abs=5e-3)
    assert bench.algorithmic_bytes_per_particle_step(0.5, 2.8) == pytest.approx(96.0 + 4.0 * n_half, rel=1e-15)
    assert bench.algorithmic_bytes_per_particle_step(0.5, 2.8) == pytest.approx(187.95, abs=5e-3)
    # unordered pairs within rc at the benchmark density: 16.36 per particle
    assert bench.pairs_within_rc_per_particle(0.5, 2.5) == pytest.approx(16.362, abs=1e-3)
    # per rebuild: binning 32, permute 104, list build 124
    assert bench.REBUILD_BYTES_PER_PARTICLE == 32.0 + 104.0 + 124.0


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("header line\nkernel_sources_sha256: %s\nhbm_bytes_per_launch: 8.25e+09\n"
                 % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == pytest.approx(8.25e9)
    f.write_text("kernel_sources_sha256: %s\nhbm_bytes_per_launch: 8.25e+09\n" % ("0" * 64))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None
