"""Host logic of bench.py (no GPU): the one-GPU guard and the gating of the
counter-measured HBM traffic on the kernel source it was taken on."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")


@pytest.fixture()
def bench():
    import bench as b
    return b


def _profile(tmp_path, sha, restart=32, traffic=3.5e9):
    p = tmp_path / "traffic.txt"
    p.write_text("# header: a comment line\n"
                 "traffic_bytes_per_launch: %.5e\n"
                 "restart: %d\n"
                 "kernel_source: paper_2608_17844_amd/csrc/gmres.hip sha256 prefix %s\n" % (traffic, restart, sha))
    return str(p)


def test_traffic_is_reported_only_for_the_kernel_source_it_was_measured_on(bench, monkeypatch, tmp_path):
    src = os.path.join(ROOT, "paper_2608_17844_amd", "csrc", "gmres.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, sha))
    assert bench.measured_traffic("arnoldi_update_dots", 32) == pytest.approx(3.5e9)
    # another restart length, another kernel class, or a changed source: no figure
    assert bench.measured_traffic("arnoldi_update_dots", 50) is None
    assert bench.measured_traffic("fft_inv_crop", 32) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, "0123456789abcdef"))
    assert bench.measured_traffic("arnoldi_update_dots", 32) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("arnoldi_update_dots", 32) is None


def test_committed_traffic_profile_matches_the_committed_kernels(bench):
    """The committed counter summary was taken on the committed gmres.hip."""
    assert bench.measured_traffic("arnoldi_update_dots", 32) is not None
