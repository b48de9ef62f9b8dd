"""Seeded synthetic inputs with the shape of the paper's workloads.

The paper measures on RTM seismic fields (Sec. 4.1, Table 1) and on stacked
images (Sec. 4.5); neither dataset is available, so these generators stand in
for them.  Every generator is a pure function of its seed (numpy PCG64) and
holds none of the codec's arithmetic: the same array feeds the CPU oracle and
the GPU path.
"""
import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def sinusoids(n, seed=0, waves=8, noise=1e-3):
    """Sum of `waves` sinusoids (frequency U[1,64] cycles over the field,
    amplitude U[0.1,1], phase U[0,2pi)) plus Gaussian noise; float32."""
    g = _rng(seed)
    f = g.uniform(1.0, 64.0, waves)
    a = g.uniform(0.1, 1.0, waves)
    ph = g.uniform(0.0, 2 * np.pi, waves)
    i = np.arange(n, dtype=np.float64) / max(n, 1)
    x = np.zeros(n, np.float64)
    for k in range(waves):
        x += a[k] * np.sin(2 * np.pi * f[k] * i + ph[k])
    x += g.normal(0.0, noise, n)
    return x.astype(np.float32)


def grf(shape, seed=0, slope=-3.0):
    """Gaussian random field with power spectrum P(k) ~ k^slope (k = 0
    removed), normalised to mean 0 and standard deviation 1; float32."""
    import scipy.fft as sfft
    g = _rng(seed)
    white = g.standard_normal(shape).astype(np.float32)
    spec = sfft.rfftn(white, workers=8)
    freqs = [np.fft.fftfreq(s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    k2 = np.zeros(spec.shape, np.float32)
    for ax, fr in enumerate(freqs):
        sh = [1] * len(shape)
        sh[ax] = fr.size
        k2 = k2 + (fr.astype(np.float32).reshape(sh)) ** 2
    k2.flat[0] = 1.0
    amp = k2 ** np.float32(slope / 4.0)  # |F| ~ k^(slope/2)
    amp.flat[0] = 0.0
    spec *= amp
    field = sfft.irfftn(spec, s=shape, workers=8).astype(np.float32)
    field -= field.mean(dtype=np.float64)
    field /= np.float32(field.std(dtype=np.float64))
    return field.astype(np.float32)


def ring_ranks(nranks=8, shape=(256, 256, 256), seed=0, sigma=1e-2):
    """Per-rank buffers of a ring Allreduce: one shared field plus a per-rank
    white perturbation; returns a list of flat float32 arrays."""
    base = grf(shape, seed).reshape(-1)
    out = []
    for r in range(nranks):
        g = _rng((seed, r + 1))
        out.append((base + g.normal(0.0, sigma, base.size).astype(np.float32))
                   .astype(np.float32))
    return out


def relative_eb(bufs, rel=1e-4):
    """Absolute bound = rel * (max - min) over all buffers, in float64."""
    lo = min(float(np.min(b)) for b in bufs)
    hi = max(float(np.max(b)) for b in bufs)
    return rel * (hi - lo)


def frames(nframes, h=2048, w=2048, seed=0, lam=50.0, src_frac=1e-4):
    """Image frames: linear background gradient + Poisson(lam) photon noise +
    sparse point sources (peak U[1e3,1e4], Gaussian PSF sigma = 1 px);
    float32 array of shape (nframes, h, w)."""
    g = _rng(seed)
    out = np.empty((nframes, h, w), np.float32)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float32)
    r = np.arange(-3, 4, dtype=np.float32)
    psf = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / 2.0).astype(np.float32)
    for f in range(nframes):
        a = g.uniform(100.0, 200.0)
        b, c = g.uniform(-0.05, 0.05, 2)
        img = (a + b * xx + c * yy).astype(np.float32)
        img += g.poisson(lam, (h, w)).astype(np.float32)
        ns = g.poisson(src_frac * h * w)
        ys = g.integers(3, h - 3, ns)
        xs = g.integers(3, w - 3, ns)
        pk = g.uniform(1e3, 1e4, ns).astype(np.float32)
        for k in range(ns):
            img[ys[k] - 3:ys[k] + 4, xs[k] - 3:xs[k] + 4] += pk[k] * psf
        out[f] = img
    return out


def sparse(n, seed=0, density=0.5):
    """Bernoulli(density) mask times N(0,1); float32."""
    g = _rng(seed)
    return (g.random(n) < density).astype(np.float32) * \
        g.standard_normal(n).astype(np.float32)


def loguniform_counts(total, nchunks, lo, hi, seed=0, multiple=1):
    """nchunks sizes drawn log-uniform in [lo, hi], rescaled to sum to total;
    the last chunk absorbs the remainder.  Returns (counts, displs) uint64."""
    g = _rng(seed)
    s = np.exp(g.uniform(np.log(lo), np.log(hi), nchunks))
    s = s / s.sum() * total
    counts = np.maximum((s // multiple).astype(np.int64) * multiple, multiple)
    counts[-1] = total - counts[:-1].sum()
    if counts[-1] <= 0:
        raise ValueError("chunk sizes do not fit the total")
    displs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return counts.astype(np.uint64), displs.astype(np.uint64)


def mixed_requests(nreq, seed=0, lo_bytes=4096, hi_bytes=16 << 20,
                   eb_lo=1e-6, eb_hi=1e-2, max_total_bytes=None):
    """Request descriptors for a batch of independent compressions:
    log-uniform byte sizes, fp32 or fp64 with p = 1/2, log-uniform absolute
    bound, GRF-like or image-like content with p = 1/2.  Returns a list of
    dicts (dtype, n, eb, kind, seed); data come from request_data()."""
    g = _rng(seed)
    reqs = []
    total = 0
    for i in range(nreq):
        nbytes = float(np.exp(g.uniform(np.log(lo_bytes), np.log(hi_bytes))))
        dtype = np.float32 if g.random() < 0.5 else np.float64
        n = max(int(nbytes) // np.dtype(dtype).itemsize, 1)
        eb = float(np.exp(g.uniform(np.log(eb_lo), np.log(eb_hi))))
        kind = "grf" if g.random() < 0.5 else "image"
        if max_total_bytes is not None and total + n * np.dtype(dtype).itemsize > max_total_bytes:
            break
        total += n * np.dtype(dtype).itemsize
        reqs.append(dict(dtype=dtype, n=n, eb=eb, kind=kind, seed=seed * 100003 + i))
    return reqs


def request_data(req):
    """Content of one request: a smooth 1D random walk of unit variance
    ("grf") or a noisy image-like row signal ("image")."""
    g = _rng(req["seed"])
    n = req["n"]
    if req["kind"] == "grf":
        steps = g.standard_normal(n)
        x = np.cumsum(steps) / np.sqrt(max(n, 1))
        x = x - x.mean()
        s = x.std()
        x = x / s if s > 0 else x
    else:
        base = g.uniform(100.0, 200.0) + g.uniform(-0.05, 0.05) * np.arange(n)
        x = (base + g.poisson(50.0, n)) / 100.0
    return x.astype(req["dtype"])


def selector_fields(seed=0, grf_shape=(64, 256, 256), n_images=2, image_hw=(1024, 1024),
                    sparse_n=1 << 22):
    """Mixed fields for the predictor selector, as (array float32, nx, eb):
    a smooth 3D GRF viewed as rows of its last axis, noisy images (the frame
    generator) and a 50%-zero sparse array tiled as 8-wide rows; each with
    eb = 1e-4 x its value range."""
    out = []
    g = grf(grf_shape, seed=seed).reshape(-1)
    out.append(g)
    for k in range(n_images):
        out.append(frames(1, image_hw[0], image_hw[1], seed=seed * 7919 + k + 1).reshape(-1))
    out.append(sparse(sparse_n, seed=seed * 7919 + 97))
    nxs = [grf_shape[-1]] + [image_hw[1]] * n_images + [8]
    res = []
    for x, nx in zip(out, nxs):
        rng_ = float(x.max()) - float(x.min())
        res.append((x.astype(np.float32), nx, 1e-4 * (rng_ if rng_ > 0 else 1.0)))
    return res


# ---- the same recipes drawn on the device (torch), for workloads too large
# to generate on the host.  Seeded with torch's device generator.

def device_grf(shape, seed, slope=-3.0):
    """The grf() recipe (P(k) ~ k^slope, k = 0 removed, mean 0, std 1) on the
    device with torch.fft; flat float32 tensor."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    spec = torch.fft.rfftn(torch.randn(shape, device="cuda", generator=g))
    k2 = torch.zeros(spec.shape, device="cuda")
    for ax, n in enumerate(shape):
        fr = torch.fft.rfftfreq(n, device="cuda") if ax == len(shape) - 1 else \
            torch.fft.fftfreq(n, device="cuda")
        sh = [1] * len(shape)
        sh[ax] = fr.numel()
        k2 = k2 + fr.view(sh) ** 2
    k2[(0,) * len(shape)] = 1.0
    amp = k2 ** (slope / 4.0)
    amp[(0,) * len(shape)] = 0.0
    f = torch.fft.irfftn(spec * amp, s=shape)
    return ((f - f.mean()) / f.std()).float().reshape(-1)


def device_frames(nframes, h=2048, w=2048, seed=0):
    """The frames() recipe (gradient background + Poisson(50) + 1e-4 point
    sources with a sigma-1 Gaussian PSF) on the device; flat float32."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    yy = torch.arange(h, device="cuda", dtype=torch.float32).view(h, 1)
    xx = torch.arange(w, device="cuda", dtype=torch.float32).view(1, w)
    out = torch.empty((nframes, h, w), device="cuda")
    r = torch.arange(-3, 4, device="cuda", dtype=torch.float32)
    psf = torch.exp(-(r.view(-1, 1) ** 2 + r.view(1, -1) ** 2) / 2)
    for f in range(nframes):
        a = 100 + 100 * torch.rand(1, device="cuda", generator=g)
        b, c = (torch.rand(2, device="cuda", generator=g) - 0.5) * 0.1
        img = a + b * xx + c * yy
        img = img + torch.poisson(torch.full((h, w), 50.0, device="cuda"), generator=g)
        ns = int(1e-4 * h * w)
        ys = torch.randint(3, h - 3, (ns,), device="cuda", generator=g)
        xs = torch.randint(3, w - 3, (ns,), device="cuda", generator=g)
        pk = 1e3 + 9e3 * torch.rand(ns, device="cuda", generator=g)
        src = torch.zeros((h, w), device="cuda")
        src.index_put_((ys, xs), pk, accumulate=True)
        img = img + torch.nn.functional.conv2d(src.view(1, 1, h, w), psf.view(1, 1, 7, 7),
                                               padding=3).view(h, w)
        out[f] = img
    return out.view(-1)


def device_selector_fields(seed=0, n_grf=10, grf_shape=(256, 256, 256), n_images=40,
                           image_hw=(2048, 2048), sparse_n=201 << 20):
    """The selector workload on the device, as (tensor, nx, eb) with eb =
    1e-4 x the field's range: n_grf smooth 3D GRFs viewed as rows of their
    last axis, n_images noisy frames, and a 50%-zero sparse array as 8-wide
    rows.  The defaults give 546 M elements (over 2^29); the fields of
    different seeds are disjoint draws."""
    import torch
    fields = [(device_grf(grf_shape, seed * 1000 + 100 + k), grf_shape[-1])
              for k in range(n_grf)]
    if n_images:
        imgs = device_frames(n_images, image_hw[0], image_hw[1],
                             seed=seed * 1000 + 3).view(n_images, -1)
        fields += [(imgs[k], image_hw[1]) for k in range(n_images)]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed * 1000 + 5)
    sp = torch.randn(sparse_n, device="cuda", generator=g) * \
        (torch.rand(sparse_n, device="cuda", generator=g) < 0.5)
    fields.append((sp, 8))
    out = []
    for x, nx in fields:
        rng_ = float(x.max() - x.min())
        out.append((x, nx, 1e-4 * (rng_ if rng_ > 0 else 1.0)))
    return out
