"""Learned predictor selector: training on the GPU and int8 export.

Per 8x8 tile an int8 network 16 -> 32 -> 3 picks the predictor (NONE, 1D or
2D Lorenzo) from 16 sampled bit-length features, instead of encoding all
three and keeping the smallest (exhaustive trial).  Labels come from
exhaustive trial (gz_tile_trial) on fields the method generates; an fp32
shadow network is trained by the library's forward/backward and Adam
kernels (gz_mlp_grad, gz_mlp_adam); the weights are then exported to int8
with power-of-two scales and loaded with gz_selector_load.  The choice is
stored in each block's header byte, so decoding never needs the network.
"""
import ctypes
import struct

import numpy as np
import torch

from . import gzccl

NIN, NH, NOUT = 16, 32, 3
NPARAM = NH * NIN + NH + NOUT * NH + NOUT
BLOB_BYTES = 756


def trial(ctx, x, nx, eb, stream=None):
    """Features int8[B,16], sizes uint32[B,3] (NONE, L1D, L2D bytes) and
    labels uint8[B] (255: RAW or ZERO tile) of every tile of x (device)."""
    n = x.numel()
    B = n // 64
    feat = torch.empty((B, 16), dtype=torch.int8, device=x.device)
    sizes = torch.empty((B, 3), dtype=torch.int32, device=x.device)
    label = torch.empty(B, dtype=torch.uint8, device=x.device)
    gzccl.check(gzccl.gz_tile_trial(ctx.h, gzccl._ptr(x), n, nx, eb, gzccl._ptr(feat),
                                    gzccl._ptr(sizes), gzccl._ptr(label),
                                    gzccl._stream(stream)), "gz_tile_trial")
    return feat, sizes, label


def init_weights(seed=0, device="cuda"):
    g = np.random.default_rng(seed)
    w = np.zeros(NPARAM, np.float32)
    w[:NH * NIN] = g.normal(0, np.sqrt(2.0 / NIN) / 16.0, NH * NIN)   # features span 0..31
    w[NH * NIN + NH:NH * NIN + NH + NOUT * NH] = g.normal(0, np.sqrt(2.0 / NH), NOUT * NH)
    return torch.from_numpy(w).to(device)


def grad(ctx, w, feat, label, stream=None):
    """Mean-loss gradient (643 floats) and loss of one batch, on the GPU."""
    g = torch.empty(NPARAM, dtype=torch.float32, device=w.device)
    loss = torch.empty(1, dtype=torch.float32, device=w.device)
    gzccl.check(gzccl.gz_mlp_grad(ctx.h, gzccl._ptr(w), gzccl._ptr(feat), gzccl._ptr(label),
                                  label.numel(), gzccl._ptr(g), gzccl._ptr(loss),
                                  gzccl._stream(stream)), "gz_mlp_grad")
    return g, loss


def train(ctx, feat, label, steps=1500, batch=16384, lr=3e-3, seed=0, log=None):
    """Adam on minibatches of the labelled tiles; returns fp32 weights."""
    keep = label < NOUT
    feat, label = feat[keep].contiguous(), label[keep].contiguous()
    N = label.numel()
    w = init_weights(seed, feat.device)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    gen = torch.Generator(device=feat.device)
    gen.manual_seed(seed)
    perm = torch.randperm(N, device=feat.device, generator=gen)
    pos = 0
    for step in range(1, steps + 1):
        if pos + batch > N:
            perm = torch.randperm(N, device=feat.device, generator=gen)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        g, loss = grad(ctx, w, feat[idx].contiguous(), label[idx].contiguous())
        gzccl.check(gzccl.gz_mlp_adam(ctx.h, gzccl._ptr(w), gzccl._ptr(g), gzccl._ptr(m),
                                      gzccl._ptr(v), step, ctypes.c_float(lr),
                                      gzccl._stream(None)), "gz_mlp_adam")
        if log and (step % 500 == 0 or step == steps):
            log(f"selector step {step}: loss {float(loss.item()):.4f}")
    return w


def _pow2_scale(maxabs, target):
    """Largest k with maxabs * 2^k <= target."""
    if maxabs <= 0:
        return 0
    return int(np.floor(np.log2(target / maxabs)))


def export_int8(w, calib_feat):
    """int8 weights with power-of-two scales: W1q = W1 2^k1, the hidden layer
    is shifted right by s so that relu(z1) * 2^(k1-s) spans 0..127 on the
    calibration features, W2q = W2 2^k2.  Returns the 756-byte blob."""
    w = np.asarray(w, np.float64)
    W1 = w[:NH * NIN].reshape(NH, NIN)
    b1 = w[NH * NIN:NH * NIN + NH]
    W2 = w[NH * NIN + NH:NH * NIN + NH + NOUT * NH].reshape(NOUT, NH)
    b2 = w[NH * NIN + NH + NOUT * NH:]
    k1 = min(_pow2_scale(np.abs(W1).max(), 127.0), 24)
    W1q = np.clip(np.rint(W1 * 2.0 ** k1), -127, 127).astype(np.int64)
    b1q = np.rint(b1 * 2.0 ** k1).astype(np.int64)
    f = np.asarray(calib_feat, np.float64)
    z1 = f @ W1.T + b1
    amax = float(np.percentile(np.maximum(z1, 0), 99.9)) if f.size else 1.0
    amax = max(amax, 1e-6)
    s = int(np.clip(k1 - _pow2_scale(amax, 127.0), 0, 24))
    hs = 2.0 ** (k1 - s)
    k2 = min(_pow2_scale(np.abs(W2).max(), 127.0), 24)
    W2q = np.clip(np.rint(W2 * 2.0 ** k2), -127, 127).astype(np.int64)
    b2q = np.rint(b2 * 2.0 ** k2 * hs).astype(np.int64)
    lim = (1 << 24) - 1
    b1q = np.clip(b1q, -lim, lim)
    b2q = np.clip(b2q, -lim, lim)
    return pack_blob(W1q, b1q, s, W2q, b2q)


def pack_blob(W1q, b1q, shift, W2q, b2q):
    out = b"GZM1" + struct.pack("<I", int(shift))
    out += np.asarray(W1q, np.int8).reshape(NH, NIN).tobytes()
    out += np.asarray(b1q, "<i4").tobytes()
    out += np.asarray(W2q, np.int8).reshape(NOUT, NH).tobytes()
    out += np.asarray(b2q, "<i4").tobytes()
    assert len(out) == BLOB_BYTES
    return out


def load(ctx, blob):
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    gzccl.check(gzccl.gz_selector_load(ctx.h, buf, len(blob)), "gz_selector_load")


def fit(ctx, fields, steps=1500, seed=0, log=None):
    """The whole training pipeline on the GPU: exhaustive-trial labels of
    every tile of `fields` ((tensor, nx, eb) on the device), Adam on the
    fp32 shadow network, int8 export calibrated on up to 50k labelled
    tiles, and loading into ctx.  Returns the blob and the label counts
    (NONE, L1D, L2D, skipped)."""
    feats, labels = [], []
    for x, nx, eb in fields:
        f, _, lab = trial(ctx, x, nx, eb)
        feats.append(f)
        labels.append(lab)
    feat = torch.cat(feats)
    lab = torch.cat(labels)
    counts = [int((lab == k).sum()) for k in range(NOUT)] + [int((lab >= NOUT).sum())]
    w = train(ctx, feat, lab, steps=steps, seed=seed, log=log)
    keep = (lab < NOUT).nonzero().view(-1)
    calib = feat[keep[:: max(1, keep.numel() // 50000)]].cpu().numpy()
    blob = export_int8(w.cpu().numpy(), calib)
    load(ctx, blob)
    return blob, counts


def tile_compress(ctx, x, nx, eb, select, out, out_bytes, threads=0, stream=None):
    """Tile-mode compression of x (device fp32, rows of nx) with selector
    `select` (0 MLP, 1 exhaustive trial, 2 always L1D) into out."""
    p = gzccl.gz_params(64, threads, 0, 1, select, nx)
    gzccl.check(gzccl.gz_compress(ctx.h, gzccl._ptr(x), x.numel(), gzccl.GZ_F32, eb,
                                  ctypes.byref(p), gzccl._ptr(out), out.numel(),
                                  gzccl._ptr(out_bytes), gzccl._stream(stream)), "gz_compress")
