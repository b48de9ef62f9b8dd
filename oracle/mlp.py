"""Float64 oracle of the selector's training math (test infrastructure).

The shadow network: z1 = W1 f + b1, h = max(z1, 0), z2 = W2 h + b2, softmax
cross-entropy against the exhaustive-trial label; samples labelled 255 (RAW
or ZERO tiles) are skipped.  Parameters are one flat vector laid out as
W1[32][16], b1[32], W2[3][32], b2[3] (643 values), the layout of the GPU
training kernels.
"""
import numpy as np

NIN, NH, NOUT = 16, 32, 3
NPARAM = NH * NIN + NH + NOUT * NH + NOUT


def unpack(w):
    w = np.asarray(w, np.float64)
    W1 = w[:NH * NIN].reshape(NH, NIN)
    b1 = w[NH * NIN:NH * NIN + NH]
    W2 = w[NH * NIN + NH:NH * NIN + NH + NOUT * NH].reshape(NOUT, NH)
    b2 = w[NH * NIN + NH + NOUT * NH:]
    return W1, b1, W2, b2


def loss_and_grad(w, feat, label):
    """Mean loss and its gradient over the labelled samples."""
    W1, b1, W2, b2 = unpack(w)
    keep = np.asarray(label) < NOUT
    f = np.asarray(feat, np.float64)[keep]
    y = np.asarray(label)[keep].astype(np.int64)
    n = f.shape[0]
    if n == 0:
        return 0.0, np.zeros(NPARAM)
    z1 = f @ W1.T + b1
    h = np.maximum(z1, 0.0)
    z2 = h @ W2.T + b2
    m = z2.max(axis=1, keepdims=True)
    e = np.exp(z2 - m)
    S = e.sum(axis=1, keepdims=True)
    p = e / S
    loss = float(np.mean(np.log(S[:, 0]) + m[:, 0] - z2[np.arange(n), y]))
    dz2 = p.copy()
    dz2[np.arange(n), y] -= 1.0
    dh = dz2 @ W2
    dz1 = dh * (z1 > 0)
    g = np.concatenate([(dz1.T @ f).ravel(), dz1.sum(0), (dz2.T @ h).ravel(), dz2.sum(0)]) / n
    return loss, g


def loss_only(w, feat, label):
    return loss_and_grad(w, feat, label)[0]
