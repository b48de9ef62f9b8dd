"""Failure handling of the kernels' bounded waits, forced from the host.

With a wait bound of zero (gz_ctx_set_wait) every wait between waves that is
not satisfied at once expires: each encoding kernel (strips and per-wave,
single streams and batches, compression and the fused step) must still
finish and report either success with the oracle's bytes or GZ_ETIMEOUT.
With the default bound restored, the same calls are clean and bit-exact.
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
    c = gz.Context(0, max_elems=1 << 25, max_requests=64)
    yield c
    c.set_wait(1_000_000)
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


EB = 1e-4
N = (1 << 22) + 1234   # 1025 superblocks: 129 rounds, 129 strips of 32768


def _calls(gz, ctx, oracle):
    """(name, run() -> list of streams as numpy arrays, expected streams)."""
    import torch
    x = synth.sinusoids(N, seed=50)
    loc = np.random.default_rng(51).normal(0, 0.2, N).astype(np.float32)
    s = oracle.compress(x, EB)
    want_c = [s]
    want_f = [oracle.fused_step(s, loc, EB)]
    X, LOC, S = dev(x), dev(loc), dev(s)

    def compress(tpb):
        def run():
            out, nb = ctx.compress(X, EB, threads=tpb)
            torch.cuda.synchronize()
            return [out[:int(nb.item())].cpu().numpy()]
        return run

    def fused(tpb):
        def run():
            out, nb = ctx.fused_reduce_step(S, LOC, EB, threads=tpb)
            torch.cuda.synchronize()
            return [out[:int(nb.item())].cpu().numpy()]
        return run

    # a uniform batch of 4 fused requests (the per-wave batch kernel by default)
    cap = gz.bound(N)
    outs = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in range(4)]
    nbs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(4)]
    items = [{"in": S, "local": LOC, "out": o, "out_bytes": b, "n": N, "in_bytes": s.size,
              "out_cap": cap, "eb": EB, "dtype": gz.GZ_F32} for o, b in zip(outs, nbs)]
    reqs = ctx.requests(items)

    def batch(tpb):
        def run():
            ctx.batch(gz.GZ_OP_FUSED, reqs, threads=tpb)
            torch.cuda.synchronize()
            return [o[:int(b.item())].cpu().numpy() for o, b in zip(outs, nbs)]
        return run

    return [("compress strips", compress(1024), want_c),
            ("compress per-wave", compress(64), want_c),
            ("fused strips", fused(1024), want_f),
            ("fused per-wave", fused(64), want_f),
            ("fused batch per-wave", batch(64), want_f * 4),
            ("fused batch strips", batch(1024), want_f * 4)]


def test_zero_wait_bound_finishes_and_reports(gz, ctx, oracle):
    statuses = []
    for name, run, want in _calls(gz, ctx, oracle):
        say("zero wait bound:", name)
        ctx.set_wait(0)
        got = run()
        st = ctx.device_status()
        statuses.append(st)
        assert st in (gz.GZ_OK, gz.GZ_ETIMEOUT), (name, st)
        if st == gz.GZ_OK:
            assert all(g.tobytes() == w.tobytes() for g, w in zip(got, want)), name
        say("  status", st)
        ctx.set_wait(1_000_000)
        ctx.reset()
        say("default bound:", name)
        got = run()
        assert ctx.device_status() == gz.GZ_OK, name
        assert all(g.tobytes() == w.tobytes() for g, w in zip(got, want)), name
    say("statuses under the zero bound", statuses)
