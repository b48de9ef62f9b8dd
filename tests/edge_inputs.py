"""Seeded inputs that drive every block kind and width edge of the GZ1 format.

Test inputs only (no codec arithmetic): values are placed on or next to the
quantisation grid t = 2*eb so that the encoder meets ZERO blocks (all +0,
all -0, |x| < eb), constant blocks (F = 0, base only), the largest in-range
quantised values (|r| = 2^29 - 32 in fp32, 2^29 - 1 in fp64), the first
out-of-range one (|r| = 2^29), widths up to F = 30, non-finite values, and
all of these across strip boundaries and in a ragged last block.
"""
import numpy as np

from paper_2308_05199_amd import synth

EB = 2.0 ** -14          # t = 2^-13 exactly, in fp32 and fp64
T = 2.0 ** -13
STRIP_EDGES = (4096, 8192, 16384, 32768, 65536)


def rmax(dt):
    """Largest |r| = |x / t| that still quantises, as an exact value of dt."""
    return float(2 ** 29 - 32) if dt == np.float32 else float(2 ** 29 - 1)


def edge_field(n, dt, seed=0):
    """A sum-of-sinusoids background with runs of special blocks; n >= 70000."""
    g = np.random.default_rng(seed)
    x = synth.sinusoids(n, seed=seed).astype(dt)
    R = rmax(dt)

    def put(lo, vals):
        vals = np.asarray(vals, dtype=np.float64)
        hi = min(n, lo + vals.size)
        x[lo:hi] = vals[:hi - lo].astype(dt)

    # ZERO: +0, -0 and |x| < eb runs, two of them across strip edges
    put(1000, np.zeros(300))
    put(2000, np.full(200, -0.0))
    put(3000, g.uniform(-0.45 * EB, 0.45 * EB, 256))
    put(STRIP_EDGES[0] - 150, np.zeros(300))
    put(STRIP_EDGES[2] - 70, np.full(140, -0.0))
    # constant runs (F = 0): on the grid, off the grid, negative, straddling
    put(5000, np.full(256, 5 * T))
    put(6000, np.full(300, 0.123456))
    put(7000, np.full(200, -3.75))
    put(STRIP_EDGES[1] - 100, np.full(200, 2.5 * T + T / 8))
    put(STRIP_EDGES[3] - 64, np.full(128, -7 * T))
    # range edges: largest in-range |r| (base only, and alternating signs:
    # residuals near 2^30, F = 30), first failing |r| = 2^29
    put(10000, np.full(128, R * T))
    put(10200, np.full(128, -R * T))
    put(10400, np.tile([R * T, -R * T], 64))
    put(10600, np.tile([R * T, 0.0, -R * T, 0.0], 32))
    put(10800, np.full(40, 2.0 ** 29 * T))
    put(11000, [-(2.0 ** 29) * T] + [0.0] * 63)
    # one in-range and one failing value per block of a run
    put(12000, np.where(np.arange(256) % 32 == 7, R * T, 0.0))
    put(12300, np.where(np.arange(256) % 64 == 50, 2.0 ** 29 * T, 1.0))
    # non-finite (quiet NaN of default payload, +-Inf) and subnormals
    x[13001] = np.nan
    x[13100] = np.inf
    x[13300] = -np.inf
    x[13500] = np.finfo(dt).tiny / 4
    # the last strip edge inside the field holds a constant run too
    if n > STRIP_EDGES[4] + 100:
        put(STRIP_EDGES[4] - 32, np.full(64, 11 * T))
    # ragged tail: alternating extreme values in the last (short) block,
    # RAW by size; the block before it constant
    tail = n % 32 if n % 32 else 32
    put(n - tail - 32, np.full(32, 9 * T))
    put(n - tail, np.tile([R * T, -R * T], tail)[:tail])
    return x


def fused_pair(n, seed=0):
    """(a, b): fp32 fields whose fused sum fl32(decode(C(a)) + b) has ZERO and
    constant blocks (both operands zero or on-grid constants there), sums
    that fail quantisation (a quiet NaN or an infinity in a, 1e30 or +-2^29 t
    in b), and ordinary blocks elsewhere."""
    g = np.random.default_rng(seed)
    a = edge_field(n, np.float32, seed)
    b = g.normal(0.0, 0.3, n).astype(np.float32)
    zero_runs = [(1000, 300), (2000, 200), (3000, 256), (STRIP_EDGES[0] - 150, 300),
                 (STRIP_EDGES[2] - 70, 140)]
    for lo, m in zero_runs:
        b[lo:lo + m] = 0.0
    # constants: a's on-grid constant runs plus an on-grid constant in b
    for lo, m, c in [(5000, 256, 3 * T), (7000, 200, -T), (STRIP_EDGES[3] - 64, 128, 2 * T)]:
        b[lo:lo + m] = np.float32(c)
    # sums outside the range: huge local values, and +-2^29 t
    b[20000:20040] = np.float32(1e30)
    b[20500:20532] = np.float32(2.0 ** 29 * T)
    b[21000:21064] = np.float32(-(2.0 ** 29) * T) - a[21000:21064]
    b[13001] = 1.0     # NaN + 1 = NaN (the quiet NaN's bits are kept)
    b[13100] = -5.0    # Inf + finite = Inf
    b[13300] = 2.0
    return a, b


def tile_edge_field(nx=64, ny=64, seed=0):
    """An nx-wide fp32 field (rows of nx values) whose 8x8 tiles cover the
    tile-mode edges: zero and -0 tiles, |x| < eb tiles, constant tiles, a
    checkerboard of +-rmax (NONE needs F = 29, L1D F = 30, L2D F = 31, which
    is RAW by size), horizontal and vertical ramps, the bilinear r*c tile,
    tiles with a NaN or an out-of-range value, and smooth tiles elsewhere."""
    g = np.random.default_rng(seed)
    x = np.zeros((ny, nx), np.float64)
    yy, xx = np.mgrid[0:ny, 0:nx]
    x[:] = np.sin(xx / 9.0) * np.cos(yy / 7.0) + g.normal(0, 1e-3, (ny, nx))
    R = rmax(np.float32)
    r, c = np.mgrid[0:8, 0:8]
    tiles = [
        np.zeros((8, 8)),
        np.full((8, 8), -0.0),
        g.uniform(-0.45 * EB, 0.45 * EB, (8, 8)),
        np.full((8, 8), 6 * T),
        np.full((8, 8), -1.2345),
        np.where((r + c) % 2 == 0, R * T, -R * T),
        np.where((r + c) % 2 == 0, -R * T, R * T),
        (3 * c) * T,
        (5 * r) * T,
        (r * c) * T,
        np.where((r == 3) & (c == 4), np.nan, 0.25),
        np.where((r == 0) & (c == 0), 2.0 ** 29 * T, 0.25),
        np.where((r == 7) & (c == 7), -(2.0 ** 29) * T, 0.0),
        np.full((8, 8), R * T),
    ]
    tpr = nx // 8
    for k, tl in enumerate(tiles):
        R0, C0 = divmod(3 * k + 1, tpr)
        x[8 * R0:8 * R0 + 8, 8 * C0:8 * C0 + 8] = tl
    return x.astype(np.float32).reshape(-1)


def forced_blob(choice):
    """Selector weights whose network always outputs `choice` (0 NONE,
    1 L1D, 2 L2D): all weights zero, output bias one-hot."""
    import struct
    out = b"GZM1" + struct.pack("<I", 0)
    out += bytes(32 * 16)
    out += np.zeros(32, "<i4").tobytes()
    out += bytes(3 * 32)
    b2 = np.zeros(3, "<i4")
    b2[choice] = 1
    out += b2.tobytes()
    return out
