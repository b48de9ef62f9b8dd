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


def test_profiles_are_of_the_current_kernels():
    """The traffic and trace summaries name the SHA-256 of the kernel source
    they were taken with; bench.py reports traffic only when it matches."""
    src = open(os.path.join(ROOT, "paper_2308_05199_amd", "csrc", "gz_kernels.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    for name in ("fused_ring_config2_traffic.txt", "ring_config2_kernel_trace.txt"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert re.search(r"[0-9a-f]{64}", text).group(0) == sha, name
        assert "rocprofv3" in text and "bench.py" in text
