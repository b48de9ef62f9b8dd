"""GPU parity of the HIP codec against the CPU oracle, through the C ABI.

Bytes, decoded values and fused sums must match the oracle bit for bit.
Every case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

from paper_2308_05199_amd import synth

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
    c = gz.Context(0, max_elems=1 << 27, max_requests=4096)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_stream(ctx, x, eb, **kw):
    import torch
    out, nb = ctx.compress(dev(x), eb, **kw)
    torch.cuda.synchronize()
    n = int(nb.item())
    return out[:n].cpu().numpy()


def assert_ok(ctx):
    assert ctx.device_status() == 0


def unless_unsupported(fn, dt, tpb):
    """fn() or None where the library reports GZ_EUNSUPPORTED for an fp64
    workgroup size: 1024 threads are built for fp32 only, 512 fp64 threads
    may need more LDS than the device gives one workgroup, and the per-wave
    encoder (threads 64) is fp32 only."""
    from paper_2308_05199_amd import gzccl
    try:
        return fn()
    except gzccl.GzError as e:
        if e.status == gzccl.GZ_EUNSUPPORTED and dt == np.float64 and (tpb >= 512 or tpb == 64):
            return None
        raise


CASES = [(np.float32, 32), (np.float32, 64), (np.float32, 128),
         (np.float64, 32), (np.float64, 64), (np.float64, 128)]


@pytest.mark.parametrize("dt,L", CASES)
@pytest.mark.parametrize("tpb", [0, 64, 128, 256, 512, 1024])   # 0 default, 64 per-wave
def test_compress_matches_oracle(ctx, oracle, dt, L, tpb):
    say("compress", dt.__name__, L, tpb)
    g = np.random.default_rng(0)
    n = 3 * 32768 + 777
    x = np.concatenate([synth.sinusoids(n - 3000, seed=1).astype(dt),
                        g.uniform(500, 1000, 3000).astype(dt)])
    for eb in (1e-4, 3e-6):
        got = unless_unsupported(lambda: gpu_stream(ctx, x, eb, block_len=L, threads=tpb), dt, tpb)
        if got is None:
            pytest.skip(f"{tpb}-thread fp64 encoding is not built or does not fit this device")
        want = oracle.compress(x, eb, block_len=L)
        assert got.tobytes() == want.tobytes()
    assert_ok(ctx)


def test_compress_sinusoid_field_2p20(ctx, oracle):
    """2^20-element sum of sinusoids + noise, eb 1e-4, L 32."""
    say("sinusoid field 2^20 compress")
    x = synth.sinusoids(1 << 20, seed=0)
    got = gpu_stream(ctx, x, 1e-4)
    want = oracle.compress(x, 1e-4)
    assert got.tobytes() == want.tobytes()
    assert_ok(ctx)


@pytest.mark.parametrize("grid", [1, 2, 7, 64, 0])
def test_bytes_independent_of_launch_shape(ctx, oracle, grid):
    say("grid", grid)
    x = synth.sinusoids(200_000, seed=2)
    want = oracle.compress(x, 1e-4, block_len=64)
    for tpb in (64, 128, 256, 512, 1024):
        got = gpu_stream(ctx, x, 1e-4, block_len=64, threads=tpb, grid=grid)
        assert got.tobytes() == want.tobytes()
    assert_ok(ctx)


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 127, 4095, 4096, 4097, 8191, 8192, 8193])
def test_small_and_ragged(ctx, oracle, n):
    say("ragged", n)
    x = synth.sinusoids(max(n, 1), seed=3)[:n]
    for L in (32, 128):
        want = oracle.compress(x, 1e-4, block_len=L)
        for tpb in (0, 64, 128, 1024):
            got = gpu_stream(ctx, x, 1e-4, block_len=L, threads=tpb)
            assert got.tobytes() == want.tobytes(), tpb
    assert_ok(ctx)


def test_special_values(ctx, oracle):
    say("specials")
    g = np.random.default_rng(4)
    x = g.normal(0, 1, 64 * 1024).astype(np.float32)
    bits = x.view(np.uint32)
    idx = g.choice(x.size, 300, replace=False)
    specials = np.array([0x7FC00000, 0x7F800000, 0xFF800000, 0x80000000, 0x00000001,
                         0x807FFFFF, 0x7F7FFFFF, 0x7FA00001], np.uint32)
    bits[idx] = specials[np.arange(idx.size) % specials.size]
    # exact ties (k + 1/2) t
    t = np.float32(2 * 2.0 ** -14)
    x[:5000] = ((np.arange(5000) - 2500 + 0.5) * t).astype(np.float32)
    for eb in (2.0 ** -14, 1e-3, 1e-40):
        want = oracle.compress(x, eb)
        for tpb in (64, 1024):
            got = gpu_stream(ctx, x, eb, threads=tpb)
            assert got.tobytes() == want.tobytes(), tpb
    assert_ok(ctx)


@pytest.mark.parametrize("dt,L", CASES)
def test_decompress_matches_oracle(ctx, oracle, dt, L):
    import torch
    say("decompress", dt.__name__, L)
    g = np.random.default_rng(5)
    n = 3 * 32768 + 1001
    x = np.concatenate([synth.sinusoids(n - 2000, seed=6).astype(dt),
                        g.uniform(500, 1000, 2000).astype(dt)])
    x[17] = np.nan
    s = oracle.compress(x, 1e-4, block_len=L)
    want = oracle.decompress(s)
    for tpb in (0, 128, 256, 512, 1024):   # 0: the per-wave decoder
        y = unless_unsupported(lambda: ctx.decompress(
            dev(s), n, dtype=torch.float32 if dt == np.float32 else torch.float64, block_len=L,
            threads=tpb), dt, tpb)
        if y is None:
            continue
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert got.view(np.uint8).tobytes() == want.view(np.uint8).tobytes()
    assert_ok(ctx)


def test_round_trip_on_gpu(ctx, oracle):
    import torch
    say("gpu round trip")
    x = synth.sinusoids(1 << 20, seed=7)
    xs = dev(x)
    s, nb = ctx.compress(xs, 1e-4)
    torch.cuda.synchronize()
    y = ctx.decompress(s, x.size, in_bytes=int(nb.item()))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    assert np.all(np.abs(y.astype(np.float64) - x) <= 1e-4)
    assert y.tobytes() == oracle.decompress(s[:int(nb.item())].cpu().numpy()).tobytes()
    assert_ok(ctx)


@pytest.mark.parametrize("L", [32, 64, 128])
def test_fused_matches_oracle(ctx, oracle, L):
    import torch
    say("fused", L)
    n = 3 * 32768 + 333
    a = synth.sinusoids(n, seed=8)
    b = np.random.default_rng(9).normal(0, 0.3, n).astype(np.float32)
    eb = 1e-4
    s = oracle.compress(a, eb, block_len=L)
    want = oracle.fused_step(s, b, eb, block_len=L)
    for tpb in (0, 64, 128, 256, 512, 1024):
        out, nb = ctx.fused_reduce_step(dev(s), dev(b), eb, block_len=L, threads=tpb)
        torch.cuda.synchronize()
        got = out[:int(nb.item())].cpu().numpy()
        assert got.tobytes() == want.tobytes(), tpb
    assert_ok(ctx)


def test_fused_minus_zero_identity(ctx):
    import torch
    say("fused -0")
    a = synth.sinusoids(100_000, seed=10)
    s, nb = ctx.compress(dev(a), 1e-4)
    torch.cuda.synchronize()
    s = s[:int(nb.item())]
    out, nb2 = ctx.fused_reduce_step(s, dev(np.full(a.size, -0.0, np.float32)), 1e-4)
    torch.cuda.synchronize()
    assert int(nb2.item()) == s.numel()
    assert torch.equal(out[:s.numel()], s)
    assert_ok(ctx)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("tpb", [0, 64])   # default (fp32: per-wave job shares; fp64: strips), per-wave
def test_scatter_matches_oracle(ctx, oracle, dt, tpb):
    import torch
    say("scatter", dt.__name__)
    n = 300_000
    x = synth.sinusoids(n, seed=11).astype(dt)
    counts, displs = synth.loguniform_counts(n, 23, 50, 40_000, seed=12)
    want, wcb, wco = oracle.scatter_compress(x, counts, displs, 1e-4, block_len=64)
    out, cb, co = ctx.scatter_compress(dev(x), counts, displs, 1e-4, block_len=64)
    torch.cuda.synchronize()
    cb, co = cb.cpu().numpy(), co.cpu().numpy()
    assert np.array_equal(cb, wcb.astype(np.int64)) and np.array_equal(co, wco.astype(np.int64))
    total = int(co[-1] + cb[-1])
    assert out[:total].cpu().numpy().tobytes() == want.tobytes()
    # batched decompression of all chunks back into one buffer
    y = ctx.scatter_decompress(out, torch.from_numpy(co).cuda(), counts, displs,
                               dtype=torch.float32 if dt == np.float32 else torch.float64,
                               block_len=64, packed_bytes=total, threads=tpb)
    torch.cuda.synchronize()
    ref = np.concatenate([oracle.decompress(want[wco[j]:wco[j] + wcb[j]])
                          for j in range(len(counts))])
    assert y.cpu().numpy().tobytes() == ref.tobytes()
    assert_ok(ctx)


def _mixed_batch(seed, nreq, max_bytes):
    reqs = synth.mixed_requests(nreq, seed=seed, lo_bytes=4096, hi_bytes=max_bytes)
    data = [synth.request_data(r) for r in reqs]
    Ls = [32, 64, 128]
    for i, r in enumerate(reqs):
        r["block_len"] = Ls[i % 3]
    return reqs, data


def test_batch_compress_decompress(ctx, oracle, gz):
    import torch
    say("batch")
    reqs, data = _mixed_batch(1, 60, 256 << 10)
    ins = [dev(d) for d in data]
    outs, nbs, items = [], [], []
    for r, x in zip(reqs, ins):
        dt = gz.GZ_F32 if r["dtype"] == np.float32 else gz.GZ_F64
        cap = gz.bound(r["n"], dt, r["block_len"])
        o = torch.empty(cap, dtype=torch.uint8, device="cuda")
        nb = torch.zeros(1, dtype=torch.int64, device="cuda")
        outs.append(o)
        nbs.append(nb)
        items.append(dict(**{"in": x}, out=o, out_bytes=nb, n=r["n"], out_cap=cap, eb=r["eb"],
                          dtype=dt, block_len=r["block_len"]))
    arr = ctx.requests(items)
    ctx.batch(gz.GZ_OP_COMPRESS, arr)
    torch.cuda.synchronize()
    streams = []
    for r, d, o, nb in zip(reqs, data, outs, nbs):
        want = oracle.compress(d, r["eb"], block_len=r["block_len"])
        got = o[:int(nb.item())].cpu().numpy()
        assert got.tobytes() == want.tobytes()
        streams.append(o[:int(nb.item())].clone())
    # batched decompression
    ys, items = [], []
    for r, s in zip(reqs, streams):
        dt = gz.GZ_F32 if r["dtype"] == np.float32 else gz.GZ_F64
        y = torch.empty(r["n"], dtype=torch.float32 if dt == gz.GZ_F32 else torch.float64,
                        device="cuda")
        ys.append(y)
        items.append(dict(**{"in": s}, out=y, n=r["n"], in_bytes=s.numel(), dtype=dt,
                          block_len=r["block_len"]))
    arr = ctx.requests(items)
    wants = [oracle.decompress(s.cpu().numpy()) for s in streams]
    for tpb in (0, 64, 512):  # default and 64: per-wave with a superblock map; 512: strips
        for y in ys:
            y.fill_(-1.0)
        ctx.batch(gz.GZ_OP_DECOMPRESS, arr, threads=tpb)
        torch.cuda.synchronize()
        for w, y in zip(wants, ys):
            assert y.cpu().numpy().tobytes() == w.tobytes(), tpb
    assert_ok(ctx)


def test_plan_and_graph_replays(ctx, oracle, gz):
    """A compress plan and a fused plan captured in one graph, replayed
    several times with eager work in between; every replay matches."""
    import torch
    say("plan/graph")
    n = 70_000
    a = [synth.sinusoids(n, seed=20 + r) for r in range(3)]
    eb = 1e-4
    A = [dev(x) for x in a]
    cap = gz.bound(n, gz.GZ_F32, 32)
    S = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in range(3)]
    NB = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(3)]
    p0 = ctx.plan(gz.GZ_OP_COMPRESS, ctx.requests([dict(**{"in": A[0]}, out=S[0], out_bytes=NB[0],
                                                         n=n, out_cap=cap, eb=eb, dtype=0)]))
    p1 = ctx.plan(gz.GZ_OP_FUSED, ctx.requests([dict(**{"in": S[0]}, local=A[1], out=S[1],
                                                      out_bytes=NB[1], n=n, in_bytes=cap,
                                                      out_cap=cap, eb=eb, dtype=0)]))
    p2 = ctx.plan(gz.GZ_OP_FUSED, ctx.requests([dict(**{"in": S[1]}, local=A[2], out=S[2],
                                                      out_bytes=NB[2], n=n, in_bytes=cap,
                                                      out_cap=cap, eb=eb, dtype=0)]))
    g = gz.Graph([p0, p1, p2])
    s0 = oracle.compress(a[0], eb)
    s1 = oracle.fused_step(s0, a[1], eb)
    s2 = oracle.fused_step(s1, a[2], eb)
    for rep in range(4):
        for s in S:
            s.zero_()
        g.launch()
        torch.cuda.synchronize()
        got = S[2][:int(NB[2].item())].cpu().numpy()
        assert got.tobytes() == s2.tobytes(), rep
        # eager work between replays
        ctx.compress(A[1], eb)
        torch.cuda.synchronize()
    assert_ok(ctx)


CORRUPTIONS = ["magic", "n", "reserved_kind", "table", "payload_total", "truncated", "pad"]


def test_job_share_batches_match_oracle(ctx, oracle, gz):
    """fp32 decoding batches of uneven jobs (sizes from a ragged part of one
    superblock to 40 superblocks, every block length): each job decoded by
    waves of its own (default and threads 64), bitwise the oracle's; a
    corrupt job sets GZ_ECORRUPT and the next batch is clean; more jobs than
    the grid has waves fall back to the (job, superblock) list."""
    import torch
    say("job shares")
    g = np.random.default_rng(60)
    ns = [int(v) for v in g.integers(100, 40 * 4096, 37)] + [4096, 4097, 1]
    Ls = [(32, 64, 128)[i % 3] for i in range(len(ns))]
    xs = [synth.sinusoids(n, seed=61 + i) for i, n in enumerate(ns)]
    streams = [oracle.compress(x, 1e-4, block_len=L) for x, L in zip(xs, Ls)]
    wants = [oracle.decompress(s) for s in streams]
    ins = [torch.from_numpy(s).cuda() for s in streams]
    ys = [torch.empty(n, device="cuda") for n in ns]
    items = [dict(**{"in": i}, out=y, n=n, in_bytes=i.numel(), dtype=gz.GZ_F32, block_len=L)
             for i, y, n, L in zip(ins, ys, ns, Ls)]
    arr = ctx.requests(items)
    for tpb in (0, 64):
        for y in ys:
            y.fill_(-1.0)
        ctx.batch(gz.GZ_OP_DECOMPRESS, arr, threads=tpb)
        torch.cuda.synchronize()
        for w, y in zip(wants, ys):
            assert y.cpu().numpy().tobytes() == w.tobytes(), tpb
    assert_ok(ctx)
    # a corrupt table word (superblock 1's offset) in a job of several superblocks
    k = next(i for i, n in enumerate(ns) if n > 3 * 4096)
    bad = streams[k].copy()
    bad[64 + 4 * 1:64 + 4 * 2] = np.frombuffer(np.uint32(0x7FFFFFF0).tobytes(), np.uint8)
    ins[k] = torch.from_numpy(bad).cuda()
    items[k] = dict(items[k], **{"in": ins[k]})
    ctx.batch(gz.GZ_OP_DECOMPRESS, ctx.requests(items), threads=64)
    torch.cuda.synchronize()
    assert ctx.device_status() == gz.GZ_ECORRUPT
    ctx.batch(gz.GZ_OP_DECOMPRESS, arr, threads=64)
    torch.cuda.synchronize()
    assert_ok(ctx)
    # 2100 one-superblock jobs: more than the 2048 waves of the grid
    ns2 = [1000 + (i % 7) * 400 for i in range(2100)]
    xs2 = [synth.sinusoids(n, seed=700 + (i % 5)) for i, n in enumerate(ns2)]
    st2 = [oracle.compress(x, 1e-4) for x in xs2]
    in2 = [torch.from_numpy(s).cuda() for s in st2]
    y2 = [torch.full((n,), -1.0, device="cuda") for n in ns2]
    items2 = [dict(**{"in": i}, out=y, n=n, in_bytes=i.numel(), dtype=gz.GZ_F32)
              for i, y, n in zip(in2, y2, ns2)]
    ctx.batch(gz.GZ_OP_DECOMPRESS, ctx.requests(items2), threads=64)
    torch.cuda.synchronize()
    for s, y in zip(st2, y2):
        assert y.cpu().numpy().tobytes() == oracle.decompress(s).tobytes()
    assert_ok(ctx)


def _corrupt(oracle, corrupt, n, seed):
    """A stream of n elements with one defect; returns (stream, readable bytes)."""
    x = synth.sinusoids(n, seed=seed)
    s = oracle.compress(x, 1e-4).copy()
    NS = -(-n // 4096)
    hoff = 64 + 4 * NS
    ib = s.size
    if corrupt == "magic":
        s[0] ^= 1
    elif corrupt == "n":
        s[8] ^= 1
    elif corrupt == "reserved_kind":
        s[hoff + 5] = 5 << 5
    elif corrupt == "table":
        s[64 + 8] ^= 4
    elif corrupt == "payload_total":
        s[24] ^= 4
    elif corrupt == "truncated":
        ib = s.size - 4
    elif corrupt == "pad":
        B = -(-n // 32)
        s[hoff + B] = 9
    if corrupt != "n":  # a different n can still be a well-formed stream
        st, _ = oracle.decompress_status(s[:ib])
        assert st == oracle.ECORRUPT
    return x, s, ib


@pytest.mark.parametrize("corrupt", CORRUPTIONS)
@pytest.mark.parametrize("tpb", [0, 512])   # per-wave and strip decoders
def test_corrupt_stream_sets_status(ctx, oracle, corrupt, tpb):
    import torch
    say("corrupt", corrupt, tpb)
    n = 20_000
    x, s, ib = _corrupt(oracle, corrupt, n, 30)
    ctx.decompress(dev(s), n, in_bytes=ib, threads=tpb)
    assert ctx.device_status() == 3  # GZ_ECORRUPT, then cleared
    y = ctx.decompress(dev(oracle.compress(x, 1e-4)), n, threads=tpb)
    torch.cuda.synchronize()
    assert ctx.device_status() == 0
    assert y.cpu().numpy().tobytes() == oracle.decompress(oracle.compress(x, 1e-4)).tobytes()


def test_argument_errors(ctx, gz):
    import ctypes
    import torch
    say("arg errors")
    x = torch.zeros(100, device="cuda")
    for eb in (0.0, -1.0, float("nan"), float("inf"), 1e-46):
        with pytest.raises(gz.GzError) as e:
            ctx.compress(x, eb)
        assert e.value.status == gz.GZ_EINVAL
    with pytest.raises(gz.GzError) as e:
        ctx.compress(x, 1e-3, out=torch.empty(100, dtype=torch.uint8, device="cuda"))
    assert e.value.status == gz.GZ_ENOSPC
    with pytest.raises(gz.GzError) as e:
        ctx.compress(x, 1e-3, block_len=48)
    assert e.value.status == gz.GZ_EINVAL
    with pytest.raises(gz.GzError) as e:
        ctx.compress(x, 1e-3, threads=384)
    assert e.value.status == gz.GZ_EINVAL
    # 1024-thread workgroups are built for fp32 1D kernels only
    with pytest.raises(gz.GzError) as e:
        ctx.compress(torch.zeros(100, dtype=torch.float64, device="cuda"), 1e-3, threads=1024)
    assert e.value.status == gz.GZ_EUNSUPPORTED
    # the per-wave kernels (threads 64): no fp64 encoder, no scatter encoder,
    # no tiles
    with pytest.raises(gz.GzError) as e:
        ctx.compress(torch.zeros(100, dtype=torch.float64, device="cuda"), 1e-3, threads=64)
    assert e.value.status == gz.GZ_EUNSUPPORTED
    with pytest.raises(gz.GzError) as e:
        ctx.scatter_compress(torch.zeros(1000, device="cuda"), [500, 500], [0, 500], 1e-3,
                             threads=64)
    assert e.value.status == gz.GZ_EUNSUPPORTED
    p64 = gz.gz_params(64, 64, 0, 1, 2, 64)
    x64 = torch.zeros(64 * 64, device="cuda")
    o64 = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    b64 = torch.zeros(1, dtype=torch.int64, device="cuda")
    st64 = gz.gz_compress(ctx.h, gz._ptr(x64), x64.numel(), gz.GZ_F32, 1e-3, ctypes.byref(p64),
                          gz._ptr(o64), o64.numel(), gz._ptr(b64), gz._stream(None))
    assert st64 == gz.GZ_EUNSUPPORTED
    xt = torch.zeros(64 * 64, device="cuda")
    cap = gz.bound(xt.numel(), gz.GZ_F32, 64)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    nb = torch.zeros(1, dtype=torch.int64, device="cuda")
    p = gz.gz_params(64, 1024, 0, 1, 2, 64)
    st = gz.gz_compress(ctx.h, gz._ptr(xt), xt.numel(), gz.GZ_F32, 1e-3, ctypes.byref(p),
                        gz._ptr(out), cap, gz._ptr(nb), gz._stream(None))
    assert st == gz.GZ_EUNSUPPORTED


def test_quantize_sampled_bit_patterns(ctx, oracle):
    """Elementwise quantisation of 2^26 bit patterns (stride sample of all
    2^32 plus dense windows around ties and range edges) equals the oracle
    for several bounds."""
    import torch
    say("quantize sweep")
    g = np.random.default_rng(31)
    bits = np.concatenate([
        (np.arange(1 << 25, dtype=np.uint64) * 128 + g.integers(0, 128, 1 << 25)).astype(np.uint32),
        g.integers(0, 1 << 32, 1 << 24, dtype=np.uint64).astype(np.uint32),
        (np.arange(1 << 23, dtype=np.uint32) + np.uint32(0x3F000000)),
        (np.arange(1 << 23, dtype=np.uint32) + np.uint32(0x4E000000)),
    ])
    x = bits.view(np.float32)
    xd = dev(x)
    for eb in (1e-4, 1e-3, 2.0 ** -14, 0.37, 3e-30):
        q, f = ctx.quantize(xd, eb)
        torch.cuda.synchronize()
        wq, wf = oracle.quantize(x, eb)
        assert np.array_equal(f.cpu().numpy().astype(bool), wf)
        assert np.array_equal(q.cpu().numpy(), wq)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("kind", ["dense", "raw"])
def test_decompress_dense_payloads(ctx, oracle, dt, kind):
    """Strips whose payload is most of (dense: ~24-bit residuals) or all of
    (raw: every block stored raw, |x / 2eb| >= 2^29) the raw size, plus a
    ragged last strip: the payload copy then needs more than one batch of
    16-byte loads per lane, fp64 strips the copy loop past the first eight
    batches, and the range ends inside a 16-byte chunk."""
    import torch
    say("decompress dense payloads", dt.__name__, kind)
    g = np.random.default_rng(31)
    n = 3 * 32768 + 333
    if kind == "dense":
        x = g.uniform(-1.0, 1.0, n).astype(dt)
    else:
        x = g.uniform(1e3, 2e3, n).astype(dt) * np.where(g.random(n) < 0.5, -1, 1).astype(dt)
    # dense: about 20 (fp32) or 27 (fp64) bits per residual, coded L1D
    eb = {"dense": 1e-6 if dt == np.float32 else 1e-8, "raw": 1e-7}[kind]
    s = oracle.compress(x, eb)
    want = oracle.decompress(s)
    least = {"dense": 0.6 if dt == np.float32 else 0.4, "raw": 0.99}[kind]
    assert s.size > least * x.nbytes
    tdt = torch.float32 if dt == np.float32 else torch.float64
    for tpb in (0, 128, 256, 512, 1024):   # 0: the per-wave decoder
        say("  threads", tpb)
        y = unless_unsupported(lambda: ctx.decompress(dev(s), n, dtype=tdt, threads=tpb), dt, tpb)
        if y is None:
            continue
        torch.cuda.synchronize()
        assert y.cpu().numpy().view(np.uint8).tobytes() == want.view(np.uint8).tobytes()
        if dt == np.float32:
            acc = dev(np.ones(n, np.float32))
            ctx.decompress_add(dev(s), acc, threads=tpb)
            torch.cuda.synchronize()
            assert acc.cpu().numpy().tobytes() == (want + np.float32(1)).tobytes()
    assert_ok(ctx)


@pytest.mark.parametrize("dt,L", CASES)
def test_wave_decoder_sizes(ctx, oracle, dt, L):
    """The default decoder (one wave per 4096-element superblock, assigned
    statically): single elements, one partial superblock, exact superblock
    multiples, a ragged last superblock, and enough superblocks that every
    wave decodes several; mixed smooth, NaN, constant, zero and raw-coded
    blocks.  Decoded values equal the oracle's bit for bit."""
    import torch
    g = np.random.default_rng(77)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    for n in (1, 33, 4095, 4096, 4097, 70001, (1 << 23) + 12345):
        say("wave decoder", dt.__name__, L, n)
        x = synth.sinusoids(n, seed=n % 97).astype(dt)
        if n > 5000:
            x[100:4300] = 0
            x[5000:5200] = dt(3.5e-3)
            x[4444] = np.nan
            x[-700:] = g.uniform(500, 1000, 700).astype(dt)
        s = oracle.compress(x, 1e-4, block_len=L)
        y = ctx.decompress(dev(s), n, dtype=tdt, block_len=L)
        torch.cuda.synchronize()
        assert y.cpu().numpy().view(np.uint8).tobytes() == \
            oracle.decompress(s).view(np.uint8).tobytes(), n
    assert_ok(ctx)


def _uniform_batch(gz, ns, eb, L, seed):
    """fp32 compress requests whose lengths share a superblock count."""
    import torch
    xs = [synth.sinusoids(n, seed=seed + i) for i, n in enumerate(ns)]
    cap = max(gz.bound(n, gz.GZ_F32, L) for n in ns)
    outs = [torch.zeros(cap, dtype=torch.uint8, device="cuda") for _ in ns]
    nbs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in ns]
    ins = [dev(x) for x in xs]
    items = [dict(**{"in": i}, out=o, out_bytes=b, n=n, out_cap=cap, eb=eb, dtype=gz.GZ_F32,
                  block_len=L) for i, o, b, n in zip(ins, outs, nbs, ns)]
    return xs, ins, outs, nbs, items, cap


@pytest.mark.parametrize("L", [32, 64, 128])
def test_wave_batches_match_oracle(ctx, oracle, gz, L):
    """Batches the per-wave encoder takes (fp32, one block length, equal
    superblock counts; here 9 superblocks, full and ragged last ones):
    compression, then the fused step on its output, by default, with
    threads 64 and on 1024-thread strips, every stream bitwise the oracle's;
    a mixed batch asked for waves is refused."""
    import torch
    ns = [9 * 4096, 9 * 4096 - 1, 8 * 4096 + 1, 8 * 4096 + 2049]
    eb = 1e-4
    xs, ins, outs, nbs, items, cap = _uniform_batch(gz, ns, eb, L, 40)
    want = [oracle.compress(x, eb, block_len=L) for x in xs]
    g = np.random.default_rng(41)
    locs = [g.normal(0, 0.3, n).astype(np.float32) for n in ns]
    want_f = [oracle.fused_step(w, l, eb, block_len=L) for w, l in zip(want, locs)]
    for tpb in (0, 64, 1024):
        say("wave batch", L, tpb)
        for o in outs:
            o.zero_()
        ctx.batch(gz.GZ_OP_COMPRESS, ctx.requests(items), threads=tpb)
        torch.cuda.synchronize()
        for w, o, b in zip(want, outs, nbs):
            assert o[:int(b.item())].cpu().numpy().tobytes() == w.tobytes(), tpb
        fo = [torch.zeros(cap, dtype=torch.uint8, device="cuda") for _ in ns]
        fb = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in ns]
        fitems = [dict(**{"in": o}, local=dev(l), out=f, out_bytes=b, n=n,
                       in_bytes=int(nb.item()), out_cap=cap, eb=eb, dtype=gz.GZ_F32,
                       block_len=L)
                  for o, l, f, b, n, nb in zip(outs, locs, fo, fb, ns, nbs)]
        ctx.batch(gz.GZ_OP_FUSED, ctx.requests(fitems), threads=tpb)
        torch.cuda.synchronize()
        for w, f, b in zip(want_f, fo, fb):
            assert f[:int(b.item())].cpu().numpy().tobytes() == w.tobytes(), tpb
    # the streams back: a uniform batch (no superblock map) on the per-wave
    # decoders, then decode-and-accumulate onto the inputs
    ys = [torch.full((n,), -1.0, device="cuda") for n in ns]
    ditems = [dict(**{"in": o}, out=y, n=n, in_bytes=int(b.item()), dtype=gz.GZ_F32, block_len=L)
              for o, y, n, b in zip(outs, ys, ns, nbs)]
    ctx.batch(gz.GZ_OP_DECOMPRESS, ctx.requests(ditems), threads=64)
    torch.cuda.synchronize()
    for w, y in zip(want, ys):
        assert y.cpu().numpy().tobytes() == oracle.decompress(w).tobytes()
    accs = [dev(x) for x in xs]
    aitems = [dict(**{"in": o}, out=a, n=n, in_bytes=int(b.item()), dtype=gz.GZ_F32, block_len=L)
              for o, a, n, b in zip(outs, accs, ns, nbs)]
    ctx.batch(gz.GZ_OP_ACCUMULATE, ctx.requests(aitems), threads=64)
    torch.cuda.synchronize()
    for w, a, x in zip(want, accs, xs):
        assert a.cpu().numpy().tobytes() == (oracle.decompress(w) + x).tobytes()
    assert_ok(ctx)
    mixed = dict(items[0])
    mixed["n"] = 3 * 4096
    with pytest.raises(gz.GzError) as e:
        ctx.batch(gz.GZ_OP_COMPRESS, ctx.requests([items[1], mixed]), threads=64)
    assert e.value.status == gz.GZ_EUNSUPPORTED


@pytest.mark.parametrize("corrupt", CORRUPTIONS)
@pytest.mark.parametrize("tpb", [0, 1024])   # per-wave and strip kernels
def test_fused_corrupt_stream_sets_status(ctx, oracle, gz, corrupt, tpb):
    """A fused step fed a corrupt stream reports GZ_ECORRUPT, and the next
    valid call is clean and bitwise the oracle's."""
    import torch
    say("fused corrupt", corrupt, tpb)
    n = 20_000
    x, s, ib = _corrupt(oracle, corrupt, n, 31)
    loc = np.random.default_rng(32).normal(0, 0.1, n).astype(np.float32)
    ctx.fused_reduce_step(dev(s), dev(loc), 1e-4, in_bytes=ib, threads=tpb)
    assert ctx.device_status() == gz.GZ_ECORRUPT
    s = oracle.compress(x, 1e-4)
    out, nb = ctx.fused_reduce_step(dev(s), dev(loc), 1e-4, threads=tpb)
    torch.cuda.synchronize()
    assert out[:int(nb.item())].cpu().numpy().tobytes() == \
        oracle.fused_step(s, loc, 1e-4).tobytes()
    assert_ok(ctx)


def test_per_wave_encoders_repeat_bit_identical(ctx, oracle, gz):
    """The per-wave encoders' offsets come from a two-level scan whose waits
    resolve in a different order on every launch: 40 launches of a fused
    plan and of a compression plan (8 ragged chunks, per-wave kernels) must
    each write the oracle's bytes every time."""
    import torch
    say("per-wave repeats")
    ns = [(1 << 20) + 3333] * 8
    eb = 1e-4
    xs, ins, outs, nbs, items, cap = _uniform_batch(gz, ns, eb, 32, 60)
    want = [oracle.compress(x, eb) for x in xs]
    g = np.random.default_rng(61)
    locs = [g.normal(0, 0.3, n).astype(np.float32) for n in ns]
    want_f = [oracle.fused_step(w, l, eb) for w, l in zip(want, locs)]
    cplan = ctx.plan(gz.GZ_OP_COMPRESS, ctx.requests(items), threads=64)
    cplan.launch()
    torch.cuda.synchronize()
    fo = [torch.zeros(cap, dtype=torch.uint8, device="cuda") for _ in ns]
    fb = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in ns]
    fitems = [dict(**{"in": o}, local=dev(l), out=f, out_bytes=b, n=n, in_bytes=cap,
                   out_cap=cap, eb=eb, dtype=gz.GZ_F32, block_len=32)
              for o, l, f, b, n in zip(outs, locs, fo, fb, ns)]
    fplan = ctx.plan(gz.GZ_OP_FUSED, ctx.requests(fitems), threads=64)
    for rep in range(40):
        for f in fo:
            f.zero_()
        fplan.launch()
        torch.cuda.synchronize()
        for w, f, b in zip(want_f, fo, fb):
            assert f[:int(b.item())].cpu().numpy().tobytes() == w.tobytes(), rep
    for rep in range(40):
        for o in outs:
            o.zero_()
        cplan.launch()
        torch.cuda.synchronize()
        for w, o, b in zip(want, outs, nbs):
            assert o[:int(b.item())].cpu().numpy().tobytes() == w.tobytes(), rep
    cplan.close()
    fplan.close()
    assert_ok(ctx)
