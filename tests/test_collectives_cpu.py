"""Pins of the collective oracles (ring Allreduce, recursive-doubling
Allreduce, decode-and-accumulate) against facts that do not come from the
oracle itself: exact sums where the codec is lossless, the error bound the
schedule allows, the schedule's size, and IEEE identities."""
import numpy as np
import pytest

from oracle import collectives as co
from paper_2308_05199_amd import synth


def integer_ranks(N, n, seed):
    g = np.random.default_rng(seed)
    return [g.integers(-3000, 3000, n).astype(np.float32) for _ in range(N)]


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_lossless_allreduce_gives_the_exact_sum_on_every_rank(oracle, N):
    """eb = 1/2 makes the step t = 1, so integer data quantise exactly and
    every stage is lossless: each rank must end with the exact sum of all N
    inputs, which fails if the schedule drops, repeats or misroutes one."""
    bufs = integer_ranks(N, 4 * 4096 + 77, seed=N)
    exact = np.sum([b.astype(np.float64) for b in bufs], axis=0)
    for x in co.redoub_allreduce(bufs, 0.5):
        assert np.array_equal(x.astype(np.float64), exact)
    assert np.array_equal(co.ring_allreduce(bufs, 0.5).astype(np.float64), exact)


@pytest.mark.parametrize("N", [2, 3, 5, 6, 8])
def test_error_bound_of_the_schedules(oracle, N):
    """Each compression adds at most eb to what it carries.  A ReDoub message
    carries its sender's accumulated error, so a participant's result holds
    the errors of every compression that fed it: r in stage 1 plus
    2^k - 1 in stage 2, N - 1 in all; the even remainder ranks add the final
    hop, N.  A ring chunk is compressed N times (1 + N - 1 fused steps).
    The fp32 additions add at most one rounding each."""
    n = 3 * 4096 + 500
    bufs = [synth.sinusoids(n, seed=10 + r) for r in range(N)]
    eb = 1e-3
    exact = np.sum([b.astype(np.float64) for b in bufs], axis=0)
    ulp = np.spacing(np.float32(np.abs(exact).max() * 2 + 1))
    r, k, part = co.redoub_schedule(N)
    res = co.redoub_allreduce(bufs, eb)
    for i, x in enumerate(res):
        hops = N if (i < 2 * r and i % 2 == 0) else N - 1
        assert np.abs(x.astype(np.float64) - exact).max() <= hops * eb + N * ulp, i
    y = co.ring_allreduce(bufs, eb)
    assert np.abs(y.astype(np.float64) - exact).max() <= N * eb + N * ulp


@pytest.mark.parametrize("N,want", [(1, 0), (2, 2), (3, 4), (4, 8), (5, 10), (6, 12),
                                    (7, 14), (8, 24)])
def test_redoub_compression_count(oracle, N, want):
    """2r (remainder in and out) + k 2^k (k steps of 2^k participants)."""
    counts = {}
    co.redoub_allreduce(integer_ranks(N, 100, 0), 0.5, counts=counts)
    assert counts["compressions"] == want


def test_schedule_partners_are_an_involution():
    for N in range(1, 17):
        r, k, part = co.redoub_schedule(N)
        assert (1 << k) <= N < (2 << k) and r == N - (1 << k)
        assert sorted(part + [2 * i for i in range(r)]) == list(range(N))
        for j in range(k):
            for p in range(1 << k):
                assert (p ^ (1 << j)) ^ (1 << j) == p and (p ^ (1 << j)) != p


def test_decompress_add_negative_zero_identity(oracle):
    """x + (-0) = x for every float, -0 and NaN included, so adding the
    stream into an accumulator of -0 reproduces the decoded values bit for
    bit (RAW blocks carry -0, NaN and infinities through)."""
    x = synth.sinusoids(20_000, seed=3)
    x[5] = -0.0
    x[100] = np.nan
    x[7000] = np.inf
    s = oracle.compress(x, 1e-4)
    got = co.decompress_add(s, np.full(x.size, -0.0, np.float32))
    assert got.tobytes() == oracle.decompress(s).tobytes()


def test_decompress_add_is_within_eb_of_the_exact_sum(oracle):
    x = synth.sinusoids(30_000, seed=4)
    acc = np.random.default_rng(5).normal(0, 1, x.size).astype(np.float32)
    got = co.decompress_add(oracle.compress(x, 1e-4), acc)
    exact = x.astype(np.float64) + acc.astype(np.float64)
    assert np.abs(got.astype(np.float64) - exact).max() <= 1e-4 + np.spacing(np.float32(8))
