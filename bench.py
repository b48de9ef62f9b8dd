"""Benchmark of the compression hot path on one MI355X.

One step = one compressed ring Reduce_scatter of 8 simulated ranks, each a
256^3 fp32 Gaussian random field (k^-3 spectrum) plus a per-rank
perturbation (sigma 1e-2), split into 8 chunks of 2^21 elements: 8 initial
compressions and 7 fused decompress -> add -> recompress steps per chunk,
eb = 1e-4 * value range, block length 32.  `value` is the uncompressed rank
data reduced per second (8 x 64 MiB per step / step time).

Also reported: compress and decompress throughput on a 2^28-element (1 GiB)
sum-of-sinusoids field, the roofline of the dominant kernel (the batched
fused step) and the CPU oracle timed on the full reduce-scatter.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N_RANKS = 8
SHAPE = (256, 256, 256)
BLOCK = 32


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-headline", action="store_true", help="skip the 1 GiB compress/decompress")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (scales profiler byte counters)")
    return ap.parse_args()


def traffic_from_profiles():
    """HBM bytes per fused launch from the committed rocprofv3 counter
    summary (None if absent or stale)."""
    path = os.path.join(ROOT, "profiles", "fused_ring_config2_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def headline(ctx, gz, torch, reps=10):
    """Compress/decompress of 2^28 fp32 values (sum of 8 sinusoids + noise,
    eb 1e-4) generated on the device."""
    import numpy as np
    n = 1 << 28
    rng = np.random.default_rng(0)
    i = torch.arange(n, device="cuda", dtype=torch.float32) / n
    x = torch.zeros(n, device="cuda", dtype=torch.float32)
    for _ in range(8):
        f, a, ph = rng.uniform(1, 64), rng.uniform(0.1, 1), rng.uniform(0, 2 * np.pi)
        x += a * torch.sin(2 * np.pi * f * i + ph)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x += 1e-3 * torch.randn(n, device="cuda", generator=g)
    del i
    out, nb = ctx.compress(x, 1e-4)
    torch.cuda.synchronize()
    cb = int(nb.item())
    y = torch.empty_like(x)
    ctx.decompress(out, n, out=y, in_bytes=cb)
    torch.cuda.synchronize()
    maxerr = float((y.double() - x.double()).abs().max().item())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        ctx.compress(x, 1e-4, out=out, out_bytes=nb)
    ev[1].record()
    for _ in range(reps):
        ctx.decompress(out, n, out=y, in_bytes=cb)
    ev[2].record()
    torch.cuda.synchronize()
    tc = ev[0].elapsed_time(ev[1]) / reps
    td = ev[1].elapsed_time(ev[2]) / reps
    raw = 4 * n
    res = {
        "workload": "2^28 fp32 sum of 8 sinusoids + N(0,1e-3), eb 1e-4, L 32",
        "ratio": raw / cb,
        "max_abs_err": maxerr,
        "compress_ms": tc, "compress_GBps": raw / tc / 1e6,
        "compress_hbm_frac": (raw + cb) / tc / 1e6 / HBM_PEAK_GBPS,
        "decompress_ms": td, "decompress_GBps": raw / td / 1e6,
        "decompress_hbm_frac": (raw + cb) / td / 1e6 / HBM_PEAK_GBPS,
    }
    del x, y, out
    torch.cuda.empty_cache()
    return res


def cpu_baseline(bufs_np, eb):
    """The oracle, unchanged, on the same reduce-scatter (all 8 chunks,
    8 operations each) on one host core."""
    import oracle
    from paper_2308_05199_amd.ring import chunk_bounds
    oracle.build(force=False)
    n = bufs_np[0].size
    t0 = time.perf_counter()
    for c, (lo, hi) in enumerate(chunk_bounds(n, N_RANKS)):
        s = oracle.compress(bufs_np[c][lo:hi], eb, block_len=BLOCK)
        for st in range(1, N_RANKS):
            s = oracle.fused_step(s, bufs_np[(c + st) % N_RANKS][lo:hi], eb, block_len=BLOCK)
    dt = time.perf_counter() - t0
    return {"value": N_RANKS * n * 4 / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "the full config-2 reduce-scatter (8 chunks x (1 compress + 7 fused "
                      f"steps), 512 MiB of rank data) on one host core, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build simulates the ring's ranks inside "
              f"one GPU's HBM); --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2308_05199_amd import gzccl, synth
    from paper_2308_05199_amd.ring import RingReduceScatter

    torch.cuda.set_device(0)
    if args.calib_copy:
        a = torch.ones(1 << 28, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 3 x 1 GiB device-to-device")
    log("generating 8 x 256^3 ranks")
    bufs_np = synth.ring_ranks(N_RANKS, SHAPE, seed=0)
    eb = synth.relative_eb(bufs_np, 1e-4)
    n = bufs_np[0].size
    ctx = gzccl.Context(0, max_elems=1 << 28, max_requests=256)
    bufs = [torch.from_numpy(b).cuda() for b in bufs_np]
    ring = RingReduceScatter(ctx, bufs, eb, block_len=BLOCK)

    # bit-exactness of chunk 0 against the oracle (outside the timed region)
    ring.run()
    torch.cuda.synchronize()
    bitexact = None
    try:
        import oracle
        oracle.build(force=False)
        lo, hi = ring.bounds[0]
        s = oracle.compress(bufs_np[0][lo:hi], eb, block_len=BLOCK)
        for st in range(1, N_RANKS):
            s = oracle.fused_step(s, bufs_np[st % N_RANKS][lo:hi], eb, block_len=BLOCK)
        streams, sizes = ring.result()
        got = streams[0][:int(sizes[0].item())].cpu().numpy()
        bitexact = got.tobytes() == s.tobytes()
    except Exception as e:  # report, never hide
        log("oracle check failed to run:", repr(e))

    # stream sizes after every step (algorithmic bytes of each launch)
    step_sizes = []
    for s in range(N_RANKS):
        ring.run_step(s)
        torch.cuda.synchronize()
        step_sizes.append(ring.sizes[s % 2].cpu().numpy().copy())
    raw_chunk = np.array([4 * (hi - lo) for lo, hi in ring.bounds], dtype=np.float64)
    fused_bytes = [float((step_sizes[s - 1] + raw_chunk + step_sizes[s]).sum())
                   for s in range(1, N_RANKS)]
    comp_bytes = float((raw_chunk + step_sizes[0]).sum())

    for _ in range(args.warmup):
        ring.run()
    torch.cuda.synchronize()

    # timed region: K steps, each launch bracketed by events on its stream
    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(N_RANKS + 1)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        evs[k][0].record()
        for s in range(N_RANKS):
            ring.run_step(s)
            evs[k][s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = np.array([[evs[k][s].elapsed_time(evs[k][s + 1]) for s in range(N_RANKS)]
                          for k in range(K)])
    ms_per_step = float(launch_ms.sum(1).mean())
    comp_ms = float(launch_ms[:, 0].mean())
    fused_ms = float(launch_ms[:, 1:].mean())
    fused_alg = float(np.mean(fused_bytes))

    # the same steps replayed as one HIP graph
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(K):
        ring.run()
    g1.record()
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / K

    st = ctx.device_status()
    streams, sizes = ring.result()
    ratio = float(raw_chunk.sum() / sizes.cpu().numpy().sum())
    head = None if args.no_headline else headline(ctx, gzccl, torch)
    cpu = None if args.no_cpu else cpu_baseline(bufs_np, eb)

    raw_step = N_RANKS * n * 4
    value = raw_step / ms_per_step / 1e6
    achieved = fused_alg / fused_ms / 1e6
    traffic = traffic_from_profiles()
    out = {
        "metric": "compress/decompress/fused-reduce GB/s and % HBM peak at eb=1e-4, bit-exact",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ring Reduce_scatter, 8 simulated ranks x 256^3 fp32 GRF "
                               "(k^-3) + N(0,1e-2) per rank, 8 chunks x 2^21, 7 fused steps "
                               "per chunk, eb = 1e-4 * range, L = 32",
                   "eb": eb, "ranks": N_RANKS, "chunk_elems": int(raw_chunk[0] // 4)},
        "bitexact_chunk0": bitexact,
        "device_status": st,
        "ratio": ratio,
        "graph_ms_per_step": graph_ms,
        "wall_ms_per_step": wall * 1e3 / K,
        "compress_launch_ms": comp_ms,
        "compress_GBps": float(raw_chunk.sum()) / comp_ms / 1e6,
        "compress_hbm_frac": comp_bytes / comp_ms / 1e6 / HBM_PEAK_GBPS,
        "fused_launch_ms": fused_ms,
        "fused_GBps": float(raw_chunk.sum()) / fused_ms / 1e6,
        "fused_hbm_frac": achieved / HBM_PEAK_GBPS,
        "headline_1GiB": head,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "kernel": "k_batch (fused decode-add-encode, 8 chunks per launch)",
                     "alg_bytes_per_launch": fused_alg,
                     "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
