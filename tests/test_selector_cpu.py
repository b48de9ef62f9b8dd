"""CPU pins of the selector pieces: the float64 training oracle against
finite differences, the int8 blob against an independent int64 forward, and
the tile-trial labels against the exhaustive definition."""
import numpy as np
import pytest

from oracle import mlp
from paper_2308_05199_amd import synth


def test_mlp_gradient_matches_finite_differences():
    g = np.random.default_rng(0)
    w = g.normal(0, 0.2, mlp.NPARAM)
    feat = g.integers(0, 32, (200, 16)).astype(np.int8)
    label = g.integers(0, 3, 200).astype(np.uint8)
    label[::17] = 255  # unlabelled tiles are skipped
    _, grad = mlp.loss_and_grad(w, feat, label)
    h = 1e-6
    for p in g.choice(mlp.NPARAM, 80, replace=False):
        e = np.zeros(mlp.NPARAM)
        e[p] = h
        fd = (mlp.loss_only(w + e, feat, label) - mlp.loss_only(w - e, feat, label)) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-6 + 1e-5 * abs(fd)


def _int64_forward(blob, f):
    """Independent reading of the blob layout and the integer network."""
    b = np.frombuffer(blob, np.uint8)
    s = int(np.frombuffer(b[4:8].tobytes(), "<u4")[0])
    W1 = b[8:520].view(np.int8).astype(np.int64).reshape(32, 16)
    b1 = b[520:648].view("<i4").astype(np.int64)
    W2 = b[648:744].view(np.int8).astype(np.int64).reshape(3, 32)
    b2 = b[744:756].view("<i4").astype(np.int64)
    acc = W1 @ f.astype(np.int64) + b1
    h = np.clip((acc + (1 << (s - 1) if s else 0)) >> s, 0, 127)
    lg = W2 @ h + b2
    return int(np.argmax(lg)), lg  # argmax takes the lowest index on ties


def test_blob_forward_matches_int64_reference(oracle):
    from paper_2308_05199_amd import selector
    g = np.random.default_rng(1)
    for trial in range(20):
        w = g.normal(0, 0.3, mlp.NPARAM).astype(np.float32)
        feats = g.integers(0, 32, (500, 16)).astype(np.int8)
        blob = selector.export_int8(w, feats)
        for f in feats[:60]:
            k, lg = oracle.mlp_forward(blob, f)
            k2, lg2 = _int64_forward(blob, f)
            assert k == k2 and np.array_equal(lg, lg2.astype(np.int32))


def test_int8_export_tracks_the_float_network(oracle):
    """The exported network picks the same class as the fp32 network on
    nearly every sample (power-of-two scales lose little)."""
    from paper_2308_05199_amd import selector
    g = np.random.default_rng(2)
    w = g.normal(0, 0.3, mlp.NPARAM)
    feats = g.integers(0, 32, (2000, 16)).astype(np.int8)
    blob = selector.export_int8(w, feats)
    W1, b1, W2, b2 = mlp.unpack(w)
    z = np.maximum(feats @ W1.T + b1, 0) @ W2.T + b2
    agree = np.mean([oracle.mlp_forward(blob, f)[0] == int(np.argmax(z[i]))
                     for i, f in enumerate(feats)])
    assert agree > 0.95


def test_tile_trial_labels_are_exhaustive_argmin(oracle):
    x, nx, eb = synth.selector_fields(3, grf_shape=(8, 64, 64), n_images=1,
                                      image_hw=(64, 128), sparse_n=1 << 14)[1]
    f, s, lab = oracle.tile_trial(x, nx, eb)
    q, fail = oracle.quantize(x, eb)
    ny = x.size // nx
    q2 = q.reshape(ny, nx)
    for b in range(0, len(lab), 7):
        R, C = divmod(b, nx // 8)
        t = q2[8 * R:8 * R + 8, 8 * C:8 * C + 8].reshape(64)
        if lab[b] != 255:
            assert lab[b] == int(np.argmin(s[b]))
            assert np.array_equal(f[b], oracle.tile_features(t))
            assert np.array_equal(s[b], oracle.tile_sizes(t))


def test_mode1_select0_uses_the_network(oracle):
    """With a blob that always answers NONE (bias only), every coded tile
    of the stream is NONE, ZERO or RAW."""
    from paper_2308_05199_amd import selector
    W1 = np.zeros((32, 16), np.int64)
    b1 = np.zeros(32, np.int64)
    W2 = np.zeros((3, 32), np.int64)
    b2 = np.array([5, 0, 0], np.int64)
    blob = selector.pack_blob(W1, b1, 0, W2, b2)
    x = synth.sinusoids(64 * 64, seed=4)
    s = oracle.compress(x, 1e-3, block_len=64, mode=1, nx=64, select=0, blob=blob)
    hdr = s[64 + 4:64 + 4 + 64]
    assert set(int(h) >> 5 for h in hdr) <= {0, 2, 7}
    y = oracle.decompress(s)
    assert np.all(np.abs(y.astype(np.float64) - x) <= 1e-3)
