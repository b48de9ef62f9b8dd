"""The binding refuses tensors the C ABI cannot take -- host tensors,
strided views, wrong dtypes, too few elements -- with GzError(GZ_EINVAL)
before any library call is made (the library only sees raw device
pointers).  Runs without a GPU: every entry point is replaced by a stub
that fails the test if reached."""
import ctypes

import pytest
import torch


@pytest.fixture()
def gz(monkeypatch):
    from paper_2308_05199_amd import gzccl

    def reached(*a, **k):
        raise AssertionError("a library call was made with a rejected argument")

    for name in gzccl.EXPORTED:
        if name not in ("gz_compress_bound", "gz_status_str"):
            monkeypatch.setattr(gzccl, name, reached)
    return gzccl


@pytest.fixture()
def ctx(gz):
    c = object.__new__(gz.Context)   # no device context: nothing may be called
    c.h = ctypes.c_void_p(0)
    c.device = 0
    return c


def rejects(gz, fn, *a, **k):
    with pytest.raises(gz.GzError) as e:
        fn(*a, **k)
    assert e.value.status == gz.GZ_EINVAL
    return str(e.value)


def test_host_tensors_are_refused(gz, ctx):
    x = torch.zeros(1000, dtype=torch.float32)
    s = torch.zeros(5000, dtype=torch.uint8)
    assert "GPU device" in rejects(gz, ctx.compress, x, 1e-4)
    assert "GPU device" in rejects(gz, ctx.decompress, s, 1000)
    assert "GPU device" in rejects(gz, ctx.fused_reduce_step, s, x, 1e-4)
    assert "GPU device" in rejects(gz, ctx.decompress_add, s, x)
    assert "GPU device" in rejects(gz, ctx.quantize, x, 1e-4)
    assert "GPU device" in rejects(gz, ctx.scatter_compress, x, [500, 500], [0, 500], 1e-4)
    off = torch.zeros(2, dtype=torch.int64)
    assert "GPU device" in rejects(gz, ctx.scatter_decompress, s, off, [500, 500], [0, 500])
    out = torch.zeros(gz.bound(1000), dtype=torch.uint8)
    nb = torch.zeros(1, dtype=torch.int64)
    assert "GPU device" in rejects(gz, gz.compress_noalloc, x, 1e-4, out, nb, None)


@pytest.fixture()
def any_device(gz, monkeypatch):
    """Host tensors stand in for device ones, so that the check under test
    (not the device check) is the one that fires."""
    monkeypatch.setattr(gz, "_on_gpu", lambda t: True)


def test_strided_views_are_refused(gz, ctx, any_device):
    x = torch.zeros(2000, dtype=torch.float32)[::2]
    assert "contiguous" in rejects(gz, ctx.compress, x, 1e-4)
    assert "contiguous" in rejects(gz, ctx.decompress_add,
                                   torch.zeros(100, dtype=torch.uint8), x)
    s = torch.zeros(10000, dtype=torch.uint8)[::2]
    assert "contiguous" in rejects(gz, ctx.decompress, s, 1000)


def test_wrong_dtypes_and_sizes_are_refused(gz, ctx, any_device):
    s = torch.zeros(5000, dtype=torch.uint8)
    assert "torch.float32" in rejects(gz, ctx.compress, torch.zeros(10, dtype=torch.int32), 1e-4)
    assert "local" in rejects(gz, ctx.fused_reduce_step, s,
                              torch.zeros(100, dtype=torch.float64), 1e-4)
    assert "out_bytes" in rejects(gz, ctx.compress, torch.zeros(10, dtype=torch.float32), 1e-4,
                                  out_bytes=torch.zeros(1, dtype=torch.int32))
    assert "stream_buf" in rejects(gz, ctx.decompress, torch.zeros(100, dtype=torch.int64), 10)
    assert "out" in rejects(gz, ctx.decompress, s, 1000, out=torch.zeros(999))
    assert "exceeds" in rejects(gz, ctx.decompress, s, 10, in_bytes=5001)
    x = torch.zeros(1000, dtype=torch.float32)
    small = torch.zeros(10, dtype=torch.uint8)
    nb = torch.zeros(1, dtype=torch.int64)
    assert "out" in rejects(gz, gz.compress_noalloc, x, 1e-4, small, nb, None)


def test_request_tensors_are_checked(gz, monkeypatch):
    f = torch.zeros(100, dtype=torch.float32)
    s = torch.zeros(1000, dtype=torch.uint8)
    nb = torch.zeros(1, dtype=torch.int64)
    base = {"in": f, "out": s, "out_bytes": nb, "n": 100, "out_cap": 1000, "eb": 1e-4,
            "dtype": gz.GZ_F32}
    for bad, word in (({"in": f[::2]}, "contiguous"),
                      ({"in": torch.zeros(100, dtype=torch.int32)}, "in"),
                      ({"in": torch.zeros(50, dtype=torch.float32)}, "fewer"),
                      ({"out_cap": 2000}, "needs"),
                      ({"local": torch.zeros(100, dtype=torch.float64)}, "local"),
                      ({"out_bytes": torch.zeros(1, dtype=torch.int32)}, "out_bytes"),
                      ):
        it = dict(base, **bad)
        with monkeypatch.context() as m:
            m.setattr(gz, "_on_gpu", lambda t: True)
            assert word in rejects(gz, gz.Context.requests, [it])
    assert "GPU device" in rejects(gz, gz.Context.requests, [base])
