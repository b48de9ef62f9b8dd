"""Compressed Allreduce of N simulated ranks on one GPU: the ring version
(Reduce_scatter, then Allgather) and the recursive-doubling version.

As in ring.py, the N ranks' buffers all live in one GPU's HBM and a "send"
hands a device stream to the receiving rank: the schedule is host logic and
every arithmetic step runs in the library's kernels.  Each step's operations
over all ranks form one batched launch, and a whole collective is one HIP
graph.
"""
import torch

from . import gzccl
from .ring import RingReduceScatter, chunk_bounds


class RingAllreduce:
    """Ring Allreduce (Sec. 3.3.3): the compressed Reduce_scatter of
    ring.py, then the Allgather stage.  The Reduce_scatter's last fused step
    is the one compression the Allgather needs; every rank then decodes all
    N chunk streams into its own output (Sec. 3.3.3: N-1 decompressions of
    received chunks, plus its own chunk, whose fp32 sum the fused step never
    writes).  All N decodes of all ranks are one batched launch."""

    def __init__(self, ctx, bufs, outs, eb, block_len=32, threads=0, grid=0, use_graph=True):
        self.rs = RingReduceScatter(ctx, bufs, eb, block_len, threads, grid, use_graph=False)
        self.N = N = len(bufs)
        n = bufs[0].numel()
        assert len(outs) == N and all(o.numel() == n and o.dtype == torch.float32 for o in outs)
        self.outs = outs
        streams, _ = self.rs.result()
        items = []
        for r in range(N):
            for c, (lo, hi) in enumerate(chunk_bounds(n, N)):
                items.append({"in": streams[c], "out": outs[r][lo:hi], "n": hi - lo,
                              "in_bytes": self.rs.caps[c], "dtype": gzccl.GZ_F32,
                              "block_len": block_len})
        self.gather = ctx.plan(gzccl.GZ_OP_DECOMPRESS, ctx.requests(items), threads=threads,
                               grid=grid)
        self.plans = self.rs.plans + [self.gather]
        self.graph = gzccl.Graph(self.plans) if use_graph else None

    def run(self, stream=None):
        if self.graph is not None:
            self.graph.launch(stream)
        else:
            for p in self.plans:
                p.launch(stream)


def redoub_schedule(N):
    """r = N - 2^k (2^k the largest power of two not above N) and the
    original ranks playing participants 0 .. 2^k-1: the odd ranks 2i+1
    (i < r), then the ranks from 2r on."""
    k = N.bit_length() - 1
    r = N - (1 << k)
    return r, k, [2 * i + 1 for i in range(r)] + list(range(2 * r, N))


class ReDoubAllreduce:
    """gZ-Allreduce (ReDoub), Sec. 3.3.4, in place on the N rank buffers.
    Stage 1: even rank 2i (i < r) compresses its whole buffer for rank
    2i+1, which decodes it and adds it to its own.  Stage 2: k steps; in
    step j every participant compresses its whole current buffer and adds
    the decoded buffer of participant p XOR 2^j to its own.  Final stage:
    rank 2i+1 compresses its result for rank 2i, which decodes it.  Each
    stage is a batched compression launch followed by a batched
    decode-and-accumulate (or decode) launch, so every compression of a step
    reads the buffers from before the step."""

    def __init__(self, ctx, bufs, eb, block_len=32, threads=0, grid=0, use_graph=True):
        self.N = N = len(bufs)
        self.n = n = bufs[0].numel()
        assert all(b.numel() == n and b.dtype == torch.float32 and b.is_cuda for b in bufs)
        self.bufs = bufs
        dev = bufs[0].device
        self.cap = cap = gzccl.bound(n, gzccl.GZ_F32, block_len)
        self.streams = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in range(N)]
        self.sizes = torch.zeros(N, dtype=torch.int64, device=dev)
        self.r, self.k, self.part = r, k, part = redoub_schedule(N)

        def comp(ranks):
            return ctx.plan(gzccl.GZ_OP_COMPRESS, ctx.requests([
                {"in": bufs[i], "out": self.streams[i], "out_bytes": self.sizes[i:i + 1],
                 "n": n, "out_cap": cap, "eb": eb, "dtype": gzccl.GZ_F32,
                 "block_len": block_len} for i in ranks]), threads=threads, grid=grid)

        def recv(op, pairs):  # (sender, receiver)
            return ctx.plan(op, ctx.requests([
                {"in": self.streams[s], "out": bufs[d], "n": n, "in_bytes": cap,
                 "dtype": gzccl.GZ_F32, "block_len": block_len} for s, d in pairs]),
                threads=threads, grid=grid)

        self.plans = []
        if r:
            self.plans.append(comp([2 * i for i in range(r)]))
            self.plans.append(recv(gzccl.GZ_OP_ACCUMULATE, [(2 * i, 2 * i + 1) for i in range(r)]))
        for j in range(k):
            self.plans.append(comp(part))
            self.plans.append(recv(gzccl.GZ_OP_ACCUMULATE,
                                   [(part[p ^ (1 << j)], part[p]) for p in range(1 << k)]))
        if r:
            self.plans.append(comp([2 * i + 1 for i in range(r)]))
            self.plans.append(recv(gzccl.GZ_OP_DECOMPRESS, [(2 * i + 1, 2 * i) for i in range(r)]))
        self.compressions = 2 * r + k * (1 << k)
        self.graph = gzccl.Graph(self.plans) if (use_graph and self.plans) else None

    def run(self, stream=None):
        if self.graph is not None:
            self.graph.launch(stream)
        else:
            for p in self.plans:
                p.launch(stream)
