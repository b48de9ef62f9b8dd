"""The allocation-free compression entry point (gz_compress_noalloc), for
callers that cannot allocate device memory, against gz_compress of a
context: byte-identical streams and sizes on consecutive calls (the second
smaller than the first, so stale contents of the shared device array would
show), every block length and element type, tile mode with the
non-learned predictors, and no change in the device's free memory."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gz():
    import torch
    from paper_2308_05199_amd import gzccl
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return gzccl


@pytest.fixture(scope="module")
def ctx(gz):
    c = gz.Context(0, max_elems=1 << 22, max_requests=16)
    yield c
    c.close()


def field(n, seed, dt):
    from paper_2308_05199_amd import synth
    x = synth.sinusoids(n, seed=seed).astype(np.float64)
    x[n // 3: n // 3 + 4096] = 0.0          # ZERO blocks
    x[n // 2: n // 2 + 300] = 7.25e-3       # constant blocks
    x[17] = np.nan                           # a RAW block
    return x.astype(dt)


def both(gz, ctx, x, eb, **kw):
    import torch
    dt = gz.GZ_F32 if x.dtype == torch.float32 else gz.GZ_F64
    L = kw.get("block_len", 32)
    cap = gz.bound(x.numel(), dt, L)
    ref, rb = ctx.compress(x, eb, **kw) if kw.get("mode", 0) == 0 else (None, None)
    if kw.get("mode", 0) == 1:
        ref = torch.empty(cap, dtype=torch.uint8, device=x.device)
        rb = torch.zeros(1, dtype=torch.int64, device=x.device)
        p = gz._params(L, kw.get("threads", 0), 0, 1, kw["select"], kw["nx"])
        gz.check(gz.gz_compress(ctx.h, gz._ptr(x), x.numel(), dt, eb, ctypes.byref(p),
                                gz._ptr(ref), cap, gz._ptr(rb), gz._stream()), "gz_compress")
    out = torch.full((cap,), 0xAB, dtype=torch.uint8, device=x.device)
    ob = torch.full((1,), -1, dtype=torch.int64, device=x.device)
    st = torch.full((1,), -1, dtype=torch.int32, device=x.device)
    gz.compress_noalloc(x, eb, out, ob, st, **kw)
    torch.cuda.synchronize()
    nb = int(rb.item())
    assert int(ob.item()) == nb
    assert int(st.item()) == gz.GZ_OK
    assert out[:nb].cpu().numpy().tobytes() == ref[:nb].cpu().numpy().tobytes()
    return nb


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("L", [32, 64, 128])
def test_noalloc_matches_context_twice(gz, ctx, dt, L):
    import torch
    for n, seed in ((5 * 32768 + 999, 3), (40_001, 4)):   # second call smaller
        say("noalloc", np.dtype(dt).name, "L", L, "n", n)
        x = torch.from_numpy(field(n, seed, dt)).cuda()
        both(gz, ctx, x, 1e-4, block_len=L)


@pytest.mark.parametrize("tpb", [128, 256, 512])
def test_noalloc_thread_counts_and_tiles(gz, ctx, tpb):
    import torch
    say("noalloc tpb", tpb)
    x = torch.from_numpy(field(3 * 32768 + 17, 5, np.float32)).cuda()
    both(gz, ctx, x, 1e-4, threads=tpb)
    nx = 256
    t = torch.from_numpy(field(nx * 8 * 40, 6, np.float32)).cuda()
    for select in (1, 2):
        say("noalloc tiles select", select, "tpb", tpb)
        both(gz, ctx, t, 1e-4, block_len=64, threads=tpb, mode=1, select=select, nx=nx)


@pytest.mark.parametrize("L", [32, 128])
def test_noalloc_per_wave_encoder_twice(gz, ctx, L):
    """threads 64: the per-wave encoder on the device-resident workspace (one
    look-back word per round of 8 superblocks), two calls in a row, the
    second smaller; bytes equal the context path's."""
    import torch
    for n, seed in ((70 * 4096 + 77, 8), (12_345, 9)):
        say("noalloc per-wave", "L", L, "n", n)
        x = torch.from_numpy(field(n, seed, np.float32)).cuda()
        both(gz, ctx, x, 1e-4, block_len=L, threads=64)


def test_noalloc_allocates_nothing_and_rejects(gz, ctx):
    import torch
    say("noalloc memory and limits")
    x = torch.from_numpy(field(1 << 20, 7, np.float32)).cuda()
    y = torch.from_numpy(field(12345, 8, np.float32)).cuda()
    cap = gz.bound(x.numel(), gz.GZ_F32, 32)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    ob = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    gz.compress_noalloc(x, 1e-4, out, ob, st)   # first call on the device: set-up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        gz.compress_noalloc(x, 1e-4, out, ob, st)
        gz.compress_noalloc(y, 1e-4, out, ob, st)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert int(st.item()) == gz.GZ_OK
    # the MLP selector needs a context's weights; oversized inputs are refused
    p = gz._params(64, 0, 0, 1, 0, 256)
    r = gz.gz_compress_noalloc(gz._ptr(x), x.numel(), gz.GZ_F32, 1e-4, ctypes.byref(p),
                               gz._ptr(out), cap, gz._ptr(ob), gz._ptr(st), gz._stream())
    assert r == gz.GZ_EINVAL
    # 32769 strips of 128 threads; real buffers of that size, so that even a
    # launch would stay in bounds
    big = 32769 * 128 * 32
    xb = torch.empty(big, dtype=torch.float32, device="cuda")
    cb = gz.bound(big, gz.GZ_F32, 32)
    ob_big = torch.empty(cb, dtype=torch.uint8, device="cuda")
    p = gz._params(32, 128, 0, 0, 0, 0)
    r = gz.gz_compress_noalloc(gz._ptr(xb), big, gz.GZ_F32, 1e-4, ctypes.byref(p),
                               gz._ptr(ob_big), cb, gz._ptr(ob), gz._ptr(st), gz._stream())
    assert r == gz.GZ_ENOSPC
