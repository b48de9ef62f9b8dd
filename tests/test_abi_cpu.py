"""Host-side checks that need no GPU: the library loads, every entry point
declared in include/gzccl.h is exported, and host validation rejects bad
arguments before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gzccl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gz_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gz_compress", "gz_decompress", "gz_fused_reduce_step", "gz_scatter_compress",
                 "gz_decompress_add", "gz_batch", "gz_plan_create", "gz_graph_create",
                 "gz_selector_load"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2308_05199_amd import gzccl
    for name in declared():
        assert hasattr(gzccl.lib, name), name
        assert name in gzccl.EXPORTED, name


def test_compress_bound_closed_form():
    from paper_2308_05199_amd import gzccl
    for n in (0, 1, 4095, 4096, 4097, 10**6):
        for dt, es in ((0, 4), (1, 8)):
            for L in (32, 64, 128):
                b = gzccl.gz_compress_bound(n, dt, L)
                assert b == 64 + 4 * -(-n // 4096) + 4 * -(-(-(-n // L)) // 4) + n * es
    assert gzccl.gz_compress_bound(10, 0, 48) == 0


def test_null_context_is_rejected_without_a_gpu():
    from paper_2308_05199_amd import gzccl
    p = gzccl.gz_params(32, 0, 0, 0, 0, 0)
    assert gzccl.gz_compress(None, None, 0, 0, 1e-4, ctypes.byref(p), None, 0, None,
                             None) == gzccl.GZ_EINVAL
    assert gzccl.gz_decompress(None, None, 0, 0, 0, None, None, None) == gzccl.GZ_EINVAL
    assert gzccl.gz_fused_reduce_step(None, None, 0, None, 0, 1e-4, None, None, 0, None,
                                      None) == gzccl.GZ_EINVAL
    assert gzccl.gz_decompress_add(None, None, 0, 0, None, None, None) == gzccl.GZ_EINVAL
    assert gzccl.gz_batch(None, 0, None, 0, None, None) == gzccl.GZ_EINVAL
    assert gzccl.gz_status_str(gzccl.GZ_ECORRUPT) == b"corrupt or mismatching stream"


def test_no_cpu_fallback_in_the_binding():
    src = open(os.path.join(ROOT, "paper_2308_05199_amd", "gzccl.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
