"""Host-side checks of bench.py and of the committed profile summaries
(no GPU needed)."""
import hashlib
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_profiles_name_their_command_and_kernel_source():
    """Each committed summary names the rocprofv3 command that made it and
    the SHA-256 of the kernel source it was taken with."""
    for name in ("fused_ring_8x256cube_traffic.txt", "ring_reduce_scatter_8x256cube_kernel_trace.txt"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert re.search(r"[0-9a-f]{64}", text), name
        assert "rocprofv3" in text and "bench.py" in text


def test_traffic_is_reported_only_for_the_profiled_kernels(tmp_path, monkeypatch):
    """bench.py reports counter traffic only while the kernel source's
    SHA-256 is the one the counters were taken with (null otherwise)."""
    sys.path.insert(0, ROOT)
    import bench
    src = open(os.path.join(ROOT, "paper_2308_05199_amd", "csrc", "gz_kernels.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_2308_05199_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2308_05199_amd" / "csrc" / "gz_kernels.hip").write_bytes(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (prof / "fused_ring_8x256cube_traffic.txt").write_text(
        f"kernel_source_sha256 = {sha}\nhbm_bytes_per_launch = 123456\n")
    assert bench.traffic_from_profiles() == 123456.0
    (prof / "fused_ring_8x256cube_traffic.txt").write_text(
        f"kernel_source_sha256 = {'0' * 64}\nhbm_bytes_per_launch = 123456\n")
    assert bench.traffic_from_profiles() is None
