"""GPU parity of decode-and-accumulate and of the two compressed Allreduce
schedules (ring: Reduce_scatter + Allgather; recursive doubling) against
the oracle, bit for bit, small and at the 8 x 256^3 workload (sampled)."""
import sys
import time

import numpy as np
import pytest

from oracle import collectives as co
from paper_2308_05199_amd import synth

pytestmark = pytest.mark.gpu

_T0 = time.time()


def say(*a):
    print(f"[case {time.time() - _T0:7.2f}s]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gz():
    import torch
    from paper_2308_05199_amd import gzccl
    assert torch.cuda.is_available()
    return gzccl


@pytest.fixture(scope="module")
def ctx(gz):
    c = gz.Context(0, max_elems=1 << 28, max_requests=4096)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def stream_with_specials(n, L, seed):
    x = np.concatenate([synth.sinusoids(n - 3000, seed=seed),
                        np.random.default_rng(seed).uniform(500, 1000, 3000).astype(np.float32)])
    x[17] = np.nan
    x[4000] = -np.inf
    x[4001] = -0.0
    return x


@pytest.mark.parametrize("L", [32, 64, 128])
@pytest.mark.parametrize("tpb", [0, 64, 128, 256, 512, 1024])   # 0 default, 64 per-wave
def test_decompress_add_matches_oracle(ctx, oracle, L, tpb):
    import torch
    say("decompress_add", L, tpb)
    n = 3 * 32768 + 1001
    x = stream_with_specials(n, L, seed=L + tpb)
    s = oracle.compress(x, 1e-4, block_len=L)
    acc = np.random.default_rng(1).normal(0, 1, n).astype(np.float32)
    acc[9] = np.nan
    want = co.decompress_add(s, acc)
    a = dev(acc)
    ctx.decompress_add(dev(s), a, block_len=L, threads=tpb)
    torch.cuda.synchronize()
    assert a.cpu().numpy().tobytes() == want.tobytes()
    assert ctx.device_status() == 0


@pytest.mark.parametrize("n", [0, 1, 31, 33, 4097, 32769])
def test_decompress_add_small_and_ragged(ctx, oracle, n):
    import torch
    say("decompress_add ragged", n)
    x = synth.sinusoids(max(n, 1), seed=2)[:n]
    s = oracle.compress(x, 1e-4)
    acc = np.linspace(-1, 1, n).astype(np.float32)
    a = dev(acc) if n else torch.zeros(0, device="cuda")
    ctx.decompress_add(dev(s), a)
    torch.cuda.synchronize()
    assert a.cpu().numpy().tobytes() == co.decompress_add(s, acc).tobytes()
    assert ctx.device_status() == 0


def test_decompress_add_corrupt_stream_leaves_acc(ctx, oracle, gz):
    import torch
    say("decompress_add corrupt")
    x = synth.sinusoids(50_000, seed=3)
    s = oracle.compress(x, 1e-4).copy()
    s[0] ^= 1  # magic
    acc = np.arange(x.size, dtype=np.float32)
    a = dev(acc)
    ctx.decompress_add(dev(s), a)
    torch.cuda.synchronize()
    assert ctx.device_status() == gz.GZ_ECORRUPT
    assert a.cpu().numpy().tobytes() == acc.tobytes()
    with pytest.raises(gz.GzError) as e:  # tile mode is not an accumulate mode
        p = gz.gz_params(64, 0, 0, 1, 2, 64)
        import ctypes
        gz.check(gz.gz_decompress_add(ctx.h, gz._ptr(dev(s)), s.size, a.numel(),
                                      ctypes.byref(p), gz._ptr(a), gz._stream(None)), "t")
    assert e.value.status == gz.GZ_EINVAL


def test_batched_accumulate_plan(ctx, oracle, gz):
    import torch
    say("batched accumulate")
    g = np.random.default_rng(4)
    ns = [int(v) for v in g.integers(1000, 200_000, 12)]
    Ls = [(32, 64, 128)[i % 3] for i in range(len(ns))]
    xs = [synth.sinusoids(n, seed=20 + i) for i, n in enumerate(ns)]
    ss = [oracle.compress(x, 1e-4, block_len=L) for x, L in zip(xs, Ls)]
    accs = [g.normal(0, 1, n).astype(np.float32) for n in ns]
    S = [dev(s) for s in ss]
    A = [dev(a) for a in accs]
    items = [{"in": S[i], "out": A[i], "n": ns[i], "in_bytes": ss[i].size,
              "dtype": gz.GZ_F32, "block_len": Ls[i]} for i in range(len(ns))]
    for tpb in (0, 64, 512):  # default (strips), per-wave, strips
        plan = ctx.plan(gz.GZ_OP_ACCUMULATE, ctx.requests(items), threads=tpb)
        for rep in range(2):  # the second launch adds the streams again
            plan.launch()
            torch.cuda.synchronize()
            for i in range(len(ns)):
                want = co.decompress_add(ss[i], accs[i])
                assert A[i].cpu().numpy().tobytes() == want.tobytes(), (tpb, rep, i)
                accs[i] = want
        plan.close()
    assert ctx.device_status() == 0


@pytest.mark.parametrize("N", [2, 3, 5, 6, 8])
def test_redoub_allreduce_matches_oracle(ctx, oracle, N):
    import torch
    from paper_2308_05199_amd.allreduce import ReDoubAllreduce
    say("redoub", N)
    n = 70_000 + 13 * N
    bufs_np = [synth.sinusoids(n, seed=40 + r) for r in range(N)]
    eb = 1e-4
    want = co.redoub_allreduce(bufs_np, eb)
    bufs = [dev(b) for b in bufs_np]
    ar = ReDoubAllreduce(ctx, bufs, eb)
    assert ar.compressions == 2 * ar.r + ar.k * (1 << ar.k)
    for rep in range(2):  # graph replays, inputs restored in between
        for b, x in zip(bufs, bufs_np):
            b.copy_(torch.from_numpy(x))
        ar.run()
        torch.cuda.synchronize()
        for i in range(N):
            assert bufs[i].cpu().numpy().tobytes() == want[i].tobytes(), (rep, i)
    assert ctx.device_status() == 0


@pytest.mark.parametrize("N", [1, 3, 8])
def test_ring_allreduce_matches_oracle(ctx, oracle, N):
    import torch
    from paper_2308_05199_amd.allreduce import RingAllreduce
    say("ring allreduce", N)
    n = 8 * 4096 * N + 123
    bufs_np = [synth.sinusoids(n, seed=60 + r) for r in range(N)]
    eb = 1e-4
    want = co.ring_allreduce(bufs_np, eb)
    bufs = [dev(b) for b in bufs_np]
    outs = [torch.empty(n, device="cuda") for _ in range(N)]
    ar = RingAllreduce(ctx, bufs, outs, eb)
    for rep in range(2):
        for o in outs:
            o.fill_(7.0)
        ar.run()
        torch.cuda.synchronize()
        for r in range(N):
            assert outs[r].cpu().numpy().tobytes() == want.tobytes(), (rep, r)
    assert ctx.device_status() == 0


def windows(n, count, width, seed):
    """Block-aligned windows [lo, lo + width): every block of the codec is
    independent, so a window of the collective equals the collective of the
    window."""
    g = np.random.default_rng(seed)
    los = sorted(set(int(v) // 4096 * 4096 for v in g.integers(0, n - width, count)))
    return [(lo, lo + width) for lo in los] + [(n - width, n)]


def test_allreduce_8x256cubed_sampled(ctx, oracle):
    """Both schedules on 8 ranks of 256^3 fp32 (the Reduce_scatter
    workload): sampled windows equal the oracle on the windows; every element
    is within the schedules' error bound of the exact sum."""
    import torch
    from paper_2308_05199_amd.allreduce import ReDoubAllreduce, RingAllreduce
    say("8 x 256^3")
    N = 8
    bufs_np = synth.ring_ranks(N, (256, 256, 256), seed=0)
    eb = synth.relative_eb(bufs_np, 1e-4)
    n = bufs_np[0].size
    exact = np.sum([b.astype(np.float64) for b in bufs_np], axis=0)
    slack = N * np.spacing(np.float32(np.abs(exact).max() * 2))
    wins = windows(n, 4, 8192, seed=1)
    bufs = [dev(b) for b in bufs_np]
    outs = [torch.empty(n, device="cuda") for _ in range(N)]
    ring = RingAllreduce(ctx, bufs, outs, eb)
    ring.run()
    torch.cuda.synchronize()
    say("ring done, status", ctx.device_status())
    for r in (0, 5):
        y = outs[r].cpu().numpy()
        assert np.abs(y.astype(np.float64) - exact).max() <= N * eb + slack
    y = outs[3].cpu().numpy()
    for lo, hi in wins:
        # the window inside its chunk: chunks are 2^21 = whole blocks
        c = lo // (n // N)
        if (hi - 1) // (n // N) != c:
            continue
        s = oracle.compress(bufs_np[c][lo:hi], eb)
        for step in range(1, N):
            s = oracle.fused_step(s, bufs_np[(c + step) % N][lo:hi], eb)
        assert y[lo:hi].tobytes() == oracle.decompress(s).tobytes(), (lo, hi)
    del ring, outs
    red = ReDoubAllreduce(ctx, bufs, eb)
    red.run()
    torch.cuda.synchronize()
    say("redoub done, status", ctx.device_status())
    got = [b.cpu().numpy() for b in bufs]
    for i in range(N):
        assert np.abs(got[i].astype(np.float64) - exact).max() <= (N - 1) * eb + slack
    for lo, hi in wins:
        want = co.redoub_allreduce([b[lo:hi] for b in bufs_np], eb)
        for i in range(N):
            assert got[i][lo:hi].tobytes() == want[i].tobytes(), (lo, hi, i)
    assert ctx.device_status() == 0
