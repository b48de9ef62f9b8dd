"""Oracle of the compressed collectives built from the codec: ring
Allreduce (Reduce_scatter then Allgather) and recursive-doubling
Allreduce, each rank's buffer a separate array.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Every lossy step is the
C oracle's compress / decompress / fused step; every addition is one fp32
addition in numpy, decoded value first.
"""
import numpy as np

from . import gzo


def decompress_add(stream, acc):
    """The reduction after a receive (Sec. 3.3.4): fl32(decoded + acc)."""
    acc = np.ascontiguousarray(acc, dtype=np.float32)
    return np.add(gzo.decompress(stream), acc, dtype=np.float32)


def chunk_bounds(n, nranks):
    """Contiguous chunk c = [c*n//N, (c+1)*n//N)."""
    return [(c * n // nranks, (c + 1) * n // nranks) for c in range(nranks)]


def ring_reduce_scatter(bufs, eb, block_len=32):
    """Sec. 3.2.3: chunk c starts at rank c with a plain compression, then
    visits ranks c+1, ..., c+N-1 (mod N), each running the fused step
    (decode, add its own chunk, encode).  Returns the N final streams;
    chunk c's ends at rank c+N-1 (mod N)."""
    N = len(bufs)
    out = []
    for c, (lo, hi) in enumerate(chunk_bounds(bufs[0].size, N)):
        s = gzo.compress(bufs[c][lo:hi], eb, block_len=block_len)
        for step in range(1, N):
            s = gzo.fused_step(s, bufs[(c + step) % N][lo:hi], eb, block_len=block_len)
        out.append(s)
    return out


def ring_allgather(streams, n):
    """Allgather stage of the ring Allreduce (Sec. 3.3.3): the one stream of
    each chunk reaches every rank, which decodes all N of them.  Every rank
    decodes the same streams, so all ranks' results are this one array."""
    N = len(streams)
    y = np.empty(n, np.float32)
    for c, (lo, hi) in enumerate(chunk_bounds(n, N)):
        y[lo:hi] = gzo.decompress(streams[c])
    return y


def ring_allreduce(bufs, eb, block_len=32):
    return ring_allgather(ring_reduce_scatter(bufs, eb, block_len), bufs[0].size)


def redoub_schedule(N):
    """The exchange pattern of recursive-doubling Allreduce with remainder
    (Sec. 3.3.4): r = N - 2^k with 2^k the largest power of two not above N.
    Returns (r, k, part) where part[p] is the original rank that plays
    rank p among the 2^k participants: the odd ranks 2i+1 (i < r) and the
    ranks i >= 2r."""
    k = N.bit_length() - 1
    r = N - (1 << k)
    part = [2 * i + 1 for i in range(r)] + list(range(2 * r, N))
    assert len(part) == 1 << k
    return r, k, part


def redoub_allreduce(bufs, eb, block_len=32, counts=None):
    """gZ-Allreduce (ReDoub), Sec. 3.3.4.  Stage 1: even rank 2i (i < r)
    compresses its whole buffer for rank 2i+1, which decodes it and adds it
    to its own.  Stage 2: in each of k steps every participant compresses its
    current buffer, the partner p XOR 2^step decodes it and adds it to its
    own (all compressions of a step read the buffers from before the step).
    Final stage: rank 2i+1 compresses its result for rank 2i, which decodes
    it.  Returns the N results; counts (a dict) receives the number of
    compressions."""
    N = len(bufs)
    x = [np.ascontiguousarray(b, dtype=np.float32).copy() for b in bufs]
    r, k, part = redoub_schedule(N)
    ncomp = 0
    for i in range(r):
        s = gzo.compress(x[2 * i], eb, block_len=block_len)
        ncomp += 1
        x[2 * i + 1] = decompress_add(s, x[2 * i + 1])
    for step in range(k):
        sent = [gzo.compress(x[part[p]], eb, block_len=block_len) for p in range(1 << k)]
        ncomp += 1 << k
        for p in range(1 << k):
            x[part[p]] = decompress_add(sent[p ^ (1 << step)], x[part[p]])
    for i in range(r):
        s = gzo.compress(x[2 * i + 1], eb, block_len=block_len)
        ncomp += 1
        x[2 * i] = gzo.decompress(s)
    if counts is not None:
        counts["compressions"] = ncomp
    return x
