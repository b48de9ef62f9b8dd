"""The boundary's ownership and concurrency rules on the GPU:

* plans take their descriptors from the context's arena, so creating and
  destroying them leaves the device's free memory unchanged; a full arena
  answers GZ_ENOSPC and a freed range is reused; plans outliving their
  context can still be destroyed;
* gz_ctx_status reads the sticky status after the context's own stream;
* two contexts on two streams, running at the same time, write the same
  bytes as one context alone (the per-stream buffers of Sec. 3.3.4: no
  shared state, no data race).
"""
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


def compress_items(gz, xs, outs, nbs, eb=1e-4):
    return [{"in": x, "out": o, "out_bytes": nb, "n": x.numel(), "out_cap": o.numel(),
             "eb": eb, "dtype": gz.GZ_F32, "block_len": 32} for x, o, nb in zip(xs, outs, nbs)]


def test_plans_allocate_nothing_and_reuse_the_arena(gz, oracle):
    import torch
    from paper_2308_05199_amd import synth
    say("plan arena")
    ctx = gz.Context(0, max_elems=1 << 20, max_requests=4)   # arena: 16 * 4 + 64 = 128 jobs
    xs_h = [synth.sinusoids(50_000 + 777 * i, seed=i) for i in range(4)]
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    outs = [torch.empty(gz.bound(x.numel()), dtype=torch.uint8, device="cuda") for x in xs]
    nbs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in xs]
    reqs = ctx.requests(compress_items(gz, xs, outs, nbs))
    warm = ctx.plan(gz.GZ_OP_COMPRESS, reqs)     # loads the kernels
    warm.launch()
    torch.cuda.synchronize()
    warm.close()
    free0 = torch.cuda.mem_get_info()[0]
    plans = [ctx.plan(gz.GZ_OP_COMPRESS, reqs) for _ in range(32)]   # 128 jobs: full
    assert torch.cuda.mem_get_info()[0] == free0
    with pytest.raises(gz.GzError) as e:
        ctx.plan(gz.GZ_OP_COMPRESS, reqs)
    assert e.value.status == gz.GZ_ENOSPC
    plans[7].close()
    again = ctx.plan(gz.GZ_OP_COMPRESS, reqs)    # reuses the freed range
    for p in (plans[0], again, plans[31]):
        for nb in nbs:
            nb.zero_()
        p.launch()
        torch.cuda.synchronize()
        for x, o, nb in zip(xs_h, outs, nbs):
            assert o[:int(nb.item())].cpu().numpy().tobytes() == oracle.compress(x, 1e-4).tobytes()
    for p in plans:
        p.close()
    again.close()
    assert torch.cuda.mem_get_info()[0] == free0
    orphan = ctx.plan(gz.GZ_OP_COMPRESS, reqs)
    assert ctx.device_status() == 0
    ctx.close()
    orphan.close()          # its context is gone: destroying it is still safe


def test_status_is_read_after_the_contexts_stream(gz):
    import torch
    from paper_2308_05199_amd import synth
    say("status on a side stream")
    ctx = gz.Context(0, max_elems=1 << 20, max_requests=4)
    side = torch.cuda.Stream()
    x = torch.from_numpy(synth.sinusoids(70_000, seed=3)).cuda()
    with torch.cuda.stream(side):
        s, nb = ctx.compress(x, 1e-4, stream=side)
        bad = s.clone()
        bad[0] ^= 1                                   # wrong magic
        ctx.decompress(bad, 70_000, stream=side)
    assert ctx.device_status(side) == gz.GZ_ECORRUPT
    assert ctx.device_status(side) == 0               # read and cleared
    ctx.close()


def test_two_contexts_on_two_streams_write_identical_bytes(gz, oracle):
    import torch
    from paper_2308_05199_amd import synth
    say("two contexts, two streams")
    n = (1 << 22) + 12345
    xh = synth.sinusoids(n, seed=11)
    lh = synth.sinusoids(n, seed=12)
    x = torch.from_numpy(xh).cuda()
    loc = torch.from_numpy(lh).cuda()
    ref_ctx = gz.Context(0, max_elems=n, max_requests=4)
    ref, rnb = ref_ctx.compress(x, 1e-4)
    torch.cuda.synchronize()
    ref = ref[:int(rnb.item())].clone()
    reff, rfb = ref_ctx.fused_reduce_step(ref, loc, 1e-4)
    torch.cuda.synchronize()
    reff = reff[:int(rfb.item())].clone()
    assert ref.cpu().numpy().tobytes() == oracle.compress(xh, 1e-4).tobytes()
    ctxs = [gz.Context(0, max_elems=n, max_requests=4) for _ in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    res = []
    torch.cuda.synchronize()
    for rep in range(3):
        outs = []
        for c, st in zip(ctxs, streams):     # both enqueued before either is waited for
            with torch.cuda.stream(st):
                o, nb = c.compress(x, 1e-4, stream=st)
                f, fb = c.fused_reduce_step(ref, loc, 1e-4, stream=st)
                outs.append((o, nb, f, fb))
        torch.cuda.synchronize()
        res.extend(outs)
    for o, nb, f, fb in res:
        assert o[:int(nb.item())].cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()
        assert f[:int(fb.item())].cpu().numpy().tobytes() == reff.cpu().numpy().tobytes()
    for c, st in zip(ctxs, streams):
        assert c.device_status(st) == 0
        c.close()
    ref_ctx.close()
