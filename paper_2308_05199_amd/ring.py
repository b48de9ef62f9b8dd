"""Compressed ring Reduce_scatter of N simulated ranks on one GPU.

Sec. 3.2.3 of the paper: the input of size D on each of N ranks is split
into N chunks; over N-1 rounds every chunk travels around the ring and each
rank it visits decompresses it, adds its own copy of that chunk and
recompresses it.  Here the N ranks' buffers all live in one GPU's HBM and a
"send" is handing the next rank the device stream: the schedule is host
logic, every arithmetic step runs in the library's kernels.

Chunk c starts at rank c with a plain compression (step 0); at step
s = 1..N-1 rank (c+s) mod N runs the fused step on chunk c.  All N chunk
operations of one step form one batched launch, and the N launches are
captured in one HIP graph.  After the last step the stream of chunk c holds
the compressed sum over all ranks, in the fixed order
((a_c + a_{c+1}) + a_{c+2}) + ... of the ring.
"""
import torch

from . import gzccl


def chunk_bounds(n, nranks):
    """Contiguous chunk c = [c*n//N, (c+1)*n//N)."""
    return [(c * n // nranks, (c + 1) * n // nranks) for c in range(nranks)]


class RingReduceScatter:
    def __init__(self, ctx, bufs, eb, block_len=32, threads=0, grid=0, use_graph=True):
        self.ctx = ctx
        self.bufs = bufs
        self.N = N = len(bufs)
        self.n = n = bufs[0].numel()
        assert all(b.numel() == n and b.dtype == torch.float32 and b.is_cuda for b in bufs)
        self.eb = eb
        self.block_len = block_len
        self.bounds = chunk_bounds(n, N)
        dev = bufs[0].device
        self.caps = [gzccl.bound(hi - lo, gzccl.GZ_F32, block_len) for lo, hi in self.bounds]
        # two stream sets, ping-pong between consecutive steps
        self.streams = [[torch.empty(cap, dtype=torch.uint8, device=dev) for cap in self.caps]
                        for _ in range(2)]
        self.sizes = [torch.zeros(N, dtype=torch.int64, device=dev) for _ in range(2)]
        self.plans = []
        for s in range(N):
            items = []
            for c, (lo, hi) in enumerate(self.bounds):
                out = self.streams[s % 2][c]
                nb = self.sizes[s % 2][c:c + 1]
                if s == 0:
                    items.append({"in": bufs[c][lo:hi], "out": out, "out_bytes": nb,
                                  "n": hi - lo, "out_cap": self.caps[c], "eb": eb,
                                  "dtype": gzccl.GZ_F32, "block_len": block_len})
                else:
                    r = (c + s) % N
                    items.append({"in": self.streams[(s - 1) % 2][c], "local": bufs[r][lo:hi],
                                  "out": out, "out_bytes": nb, "n": hi - lo,
                                  "in_bytes": self.caps[c], "out_cap": self.caps[c], "eb": eb,
                                  "dtype": gzccl.GZ_F32, "block_len": block_len})
            op = gzccl.GZ_OP_COMPRESS if s == 0 else gzccl.GZ_OP_FUSED
            self.plans.append(ctx.plan(op, ctx.requests(items), threads=threads, grid=grid))
        self.graph = gzccl.Graph(self.plans) if use_graph else None

    @property
    def final_set(self):
        return (self.N - 1) % 2

    def run(self, stream=None):
        if self.graph is not None:
            self.graph.launch(stream)
        else:
            for p in self.plans:
                p.launch(stream)

    def run_step(self, s, stream=None):
        """Launches step s alone (0 = initial compressions)."""
        self.plans[s].launch(stream)

    def result(self):
        """(streams, sizes) of the reduced chunks after run(); chunk c is
        owned by rank (c + N - 1) mod N."""
        k = self.final_set
        return self.streams[k], self.sizes[k]

    def owner(self, c):
        return (c + self.N - 1) % self.N
