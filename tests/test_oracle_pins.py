"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed independently: bytes
worked out by hand from the format definition (tests/golden), closed forms,
invariants that hold for any correct codec, and brute force on tiny inputs.
"""
import json
import os
import struct

import numpy as np
import pytest

from paper_2308_05199_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gz1_worked_examples.json")
T13 = np.float32(2.0 ** -13)
EB14 = 2.0 ** -14


def _golden():
    with open(GOLDEN) as f:
        g = json.load(f)
    return {k: v for k, v in g.items() if not k.startswith("_")}


def _input_of(case):
    x = np.asarray(case["q"], np.float32) * T13
    for i in case["nan_at"]:
        x[i] = np.frombuffer(struct.pack("<I", 0x7FC00000), np.float32)[0]
    return x


def _expected_stream(case, x):
    n = x.size
    L = case["L"]
    payload = b""
    if "payload_raw" in case:
        for b in case["payload_raw"]:
            payload += x[b * L:(b + 1) * L].tobytes()
    else:
        payload = b"".join(struct.pack("<I", int(w, 16)) for w in case["payload_words"])
    hdr = b"GZC1" + struct.pack("<HBB", 1, 0, {32: 5, 64: 6, 128: 7}[L])
    hdr += struct.pack("<QdQIII", n, EB14, len(payload), case["mode"], case["nx"], 4096)
    hdr += b"\0" * (64 - len(hdr))
    table = b"".join(struct.pack("<I", v) for v in case["table"])
    heads = bytes(int(h, 16) for h in case["headers"])
    heads += b"\0" * ((-len(heads)) % 4)
    return hdr + table + heads + payload


@pytest.mark.parametrize("name", sorted(_golden()))
def test_worked_example_bytes(oracle, name):
    case = _golden()[name]
    x = _input_of(case)
    s = oracle.compress(x, EB14, block_len=case["L"], mode=case["mode"],
                        nx=case["nx"], select=case["select"])
    assert s.tobytes() == _expected_stream(case, x)
    y = oracle.decompress(s)
    fin = np.isfinite(x)
    assert np.array_equal(y[fin], x[fin])          # exact multiples of t
    assert np.array_equal(y.view(np.uint32)[~fin], x.view(np.uint32)[~fin])
    if "tile_sizes" in case:
        q = np.asarray(case["q"], np.int32)
        assert list(oracle.tile_sizes(q)) == case["tile_sizes"]


def test_quantize_closed_form(oracle):
    """q = rint(x/t) in float32 and x' = (float)q * t, compared with numpy's
    own IEEE float32 division and rint (a different implementation)."""
    g = np.random.default_rng(1)
    x = np.concatenate([g.normal(0, 3, 50000), g.uniform(-1e4, 1e4, 50000)]).astype(np.float32)
    for eb in (1e-4, 1e-3, 2.0 ** -14, 0.37):
        t = np.float32(2.0 * eb)
        q, fail = oracle.quantize(x, eb)
        r = x / t
        ok = np.abs(r.astype(np.float64)) <= 536870911.0
        qr = np.rint(r[ok]).astype(np.int32)
        xh = qr.astype(np.float32) * t
        good = np.abs(x[ok].astype(np.float64) - xh.astype(np.float64)) <= eb
        assert np.array_equal(fail[ok], ~good)
        assert np.array_equal(q[ok][good], qr[good])
        assert fail[~ok].all()


def test_quantize_ties_to_even(oracle):
    """x = (k + 1/2) t is an exact tie: rint goes to the even neighbour."""
    k = np.arange(-1000, 1000)
    x = ((k + 0.5) * 2.0 ** -13).astype(np.float32)
    q, fail = oracle.quantize(x, EB14)
    even = np.where(k % 2 == 0, k, k + 1)
    assert not fail.any()
    assert np.array_equal(q, even)


def test_quantize_specials(oracle):
    bits = np.array([0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000,
                     0x00000001, 0x807FFFFF, 0x7F7FFFFF], np.uint32)
    x = bits.view(np.float32)
    q, fail = oracle.quantize(x, 1e-3)
    assert list(fail) == [False, False, True, True, True, False, False, True]
    assert q[0] == 0 and q[1] == 0 and q[5] == 0 and q[6] == 0


def test_quantize_range_limit(oracle):
    """|r| <= 2^29 - 1 is encodable; the next representable quotient fails."""
    t = 2.0 ** -13
    x = np.array([(2 ** 29 - 32) * t, 2 ** 29 * t, -(2 ** 29 - 32) * t, -(2 ** 29) * t],
                 np.float32)
    q, fail = oracle.quantize(x, EB14)
    assert list(fail) == [False, True, False, True]
    assert q[0] == 2 ** 29 - 32 and q[2] == -(2 ** 29 - 32)


def test_quantize_fp64(oracle):
    g = np.random.default_rng(2)
    x = g.normal(0, 10, 20000)
    eb = 1e-5
    q, fail = oracle.quantize(x, eb)
    t = 2.0 * eb
    qr = np.rint(x / t)
    good = np.abs(x - qr * t) <= eb
    assert np.array_equal(fail, ~good)
    assert np.array_equal(q[good], qr[good].astype(np.int32))


def _decode_q(stream, x, eb, oracle):
    """Quantised values implied by a decoded array (exact for non-RAW)."""
    y = oracle.decompress(stream)
    t = np.float32(2 * eb) if x.dtype == np.float32 else 2 * eb
    return y, np.rint(y / t)


@pytest.mark.parametrize("L", [32, 64, 128])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_round_trip_error_bound(oracle, L, dt):
    """Invariant: every decoded value is within eb of its input (RAW blocks
    exactly equal), for noisy data, data near ulp(x) and a ragged tail."""
    g = np.random.default_rng(3)
    n = 3 * 4096 + 777
    x = np.concatenate([synth.sinusoids(n - 2000, seed=5).astype(dt),
                        (g.uniform(500, 1000, 2000)).astype(dt)])
    for eb in (1e-4, 1e-3, 3e-5):
        s = oracle.compress(x, eb, block_len=L)
        y = oracle.decompress(s)
        assert y.dtype == x.dtype and y.size == x.size
        assert np.all(np.abs(x.astype(np.float64) - y.astype(np.float64)) <= eb)


def test_raw_iff_violation_brute_force(oracle):
    """Brute force on tiny blocks: a block is RAW exactly when some element
    would miss the bound after quantise/reconstruct (recomputed here with
    numpy float32 arithmetic)."""
    g = np.random.default_rng(4)
    eb = 1e-3
    t = np.float32(2 * eb)
    for trial in range(300):
        x = (g.uniform(500, 1100, 32)).astype(np.float32)
        if trial % 3 == 0:
            x = (g.normal(0, 1, 32)).astype(np.float32)
        s = oracle.compress(x, eb)
        hb = s[68]
        r = x / t
        qr = np.rint(r)
        xh = qr.astype(np.int32).astype(np.float32) * t
        bad = np.abs(x.astype(np.float64) - xh.astype(np.float64)) > eb
        assert (hb >> 5 == 7) == bool(bad.any())


def _blocks(stream):
    info = None
    n = struct.unpack_from("<Q", stream, 8)[0]
    L = 1 << int(stream[7])
    B = -(-n // L)
    NS = -(-n // 4096)
    hdr = [int(h) for h in stream[64 + 4 * NS: 64 + 4 * NS + B]]
    return n, L, B, NS, hdr, info


def test_width_minimal_brute_force(oracle):
    """F is the smallest width that holds every residual: recomputed from the
    decoded q by brute force over all widths."""
    g = np.random.default_rng(5)
    x = np.cumsum(g.normal(0, 1, 32 * 200)).astype(np.float32) * np.float32(0.01)
    eb = 1e-3
    s = oracle.compress(x, eb)
    n, L, B, NS, hdr, _ = _blocks(s)
    t = np.float32(2 * eb)
    y = oracle.decompress(s)
    q = np.rint(y / t).astype(np.int64).reshape(B, L)
    for b in range(B):
        kind, F = hdr[b] >> 5, hdr[b] & 31
        if kind != 1:
            continue
        d = np.diff(q[b])
        m = int(np.max(np.abs(d))) if d.size else 0
        widths = [w for w in range(32) if m < (1 << w)]
        assert F == widths[0]


def test_constant_block_packs_to_zero_width(oracle):
    x = np.full(32 * 9, 0.731, np.float32)
    s = oracle.compress(x, 1e-4)
    _, _, B, _, hdr, _ = _blocks(s)
    assert all(h == 0x20 for h in hdr)
    assert len(s) == 64 + 4 + 12 + 9 * 4


def test_zero_closed_form(oracle):
    """eb >= max|x| (1 + 2^-20): every q is 0, every block is ZERO, and the
    stream is header + zero table + zero header bytes."""
    g = np.random.default_rng(6)
    for n in (1, 31, 4096, 5000, 12345):
        x = g.normal(0, 1, n).astype(np.float32)
        eb = float(np.max(np.abs(x))) * (1 + 2 ** -20)
        s = oracle.compress(x, eb, block_len=64)
        NS, B = -(-n // 4096), -(-n // 64)
        assert len(s) == 64 + 4 * NS + 4 * (-(-B // 4))
        assert not s[64:].any()
        assert not oracle.decompress(s).view(np.uint32).any()  # +0.0 everywhere


def test_table_is_cumsum_of_sizes(oracle):
    """Closed form: superblock entries = exclusive cumulative sum of the block
    sizes implied by the header bytes, at every 4096-element boundary."""
    x = synth.sinusoids(4096 * 5 + 100, seed=7)
    for L in (32, 64, 128):
        s = oracle.compress(x, 1e-4, block_len=L)
        n, L_, B, NS, hdr, _ = _blocks(s)
        sizes = []
        for b in range(B):
            kind, F = hdr[b] >> 5, hdr[b] & 31
            m = min(L, n - b * L)
            sizes.append({0: 0, 1: 4 + ((F + 1) * L // 8 if F else 0), 7: 4 * m}[kind])
        off = np.concatenate([[0], np.cumsum(sizes)])
        table = np.frombuffer(s[64:64 + 4 * NS].tobytes(), np.uint32)
        per = 4096 // L
        assert np.array_equal(table.astype(np.int64) * 4, off[::per][:NS])
        assert struct.unpack_from("<Q", s, 24)[0] == off[-1]
        assert len(s) == 64 + 4 * NS + 4 * (-(-B // 4)) + off[-1]


def test_idempotence(oracle):
    """C(D(C(x))) == C(x) byte for byte when every |q| < 2^22."""
    for dt in (np.float32, np.float64):
        x = synth.sinusoids(20000, seed=8).astype(dt)
        for L in (32, 128):
            s = oracle.compress(x, 1e-4, block_len=L)
            s2 = oracle.compress(oracle.decompress(s), 1e-4, block_len=L)
            assert s.tobytes() == s2.tobytes()


def test_decode_of_encode_is_q(oracle):
    """decode(encode(x)) == (T)q * t with q from the quantiser."""
    x = synth.sinusoids(9000 * 32, seed=9)
    eb = 1e-4
    q, fail = oracle.quantize(x, eb)
    y = oracle.decompress(oracle.compress(x, eb))
    raw = np.repeat(fail.reshape(-1, 32).any(1), 32)
    assert 0 < raw.mean() < 0.5          # rounding near ulp(x) forces some RAW blocks
    assert np.array_equal(y[~raw], q[~raw].astype(np.float32) * np.float32(2 * eb))
    assert np.array_equal(y[raw].view(np.uint32), x[raw].view(np.uint32))


def test_empty_input(oracle):
    s = oracle.compress(np.zeros(0, np.float32), 1e-4)
    assert len(s) == 64
    assert oracle.decompress(s).size == 0


def test_fused_minus_zero_is_identity(oracle):
    """A local buffer of -0.0 leaves the stream unchanged (x' + -0 = x' and
    re-encoding x' is idempotent)."""
    x = synth.sinusoids(30000, seed=10)
    s = oracle.compress(x, 1e-4)
    out = oracle.fused_step(s, np.full(x.size, -0.0, np.float32), 1e-4)
    assert out.tobytes() == s.tobytes()


def test_fused_is_numpy_chain(oracle):
    """The fused step equals decode -> numpy float32 add -> encode."""
    g = np.random.default_rng(11)
    a = synth.sinusoids(10000, seed=11)
    b = g.normal(0, 0.5, a.size).astype(np.float32)
    eb = 1e-4
    s = oracle.compress(a, eb)
    y = oracle.decompress(s) + b
    assert oracle.fused_step(s, b, eb).tobytes() == oracle.compress(y, eb).tobytes()


def test_ring_error_accumulates_k_eb(oracle):
    """Sec. 3.3.3 (accuracy loss): every compression adds at most eb, so after
    k fused steps the value sent on is within (k+1) eb of the exact sum, up to
    the float32 rounding of the k additions."""
    nr = 6
    bufs = [synth.sinusoids(8192, seed=20 + r) for r in range(nr)]
    eb = 1e-4
    s = oracle.compress(bufs[0], eb)
    exact = bufs[0].astype(np.float64)
    rho = np.zeros(8192)
    for k in range(1, nr):
        xprev = oracle.decompress(s)
        y = xprev + bufs[k]
        rho += np.spacing(np.abs(y)).astype(np.float64) / 2
        s = oracle.fused_step(s, bufs[k], eb)
        exact += bufs[k]
        err = np.abs(oracle.decompress(s).astype(np.float64) - exact)
        assert np.all(err <= (k + 1) * eb + rho + 1e-12)


def test_ring_error_is_unbiased(oracle):
    """Sec. 3.3.3: the expected accumulated error is zero.  The mean signed
    error over many elements is far below eb."""
    bufs = [synth.sinusoids(1 << 16, seed=40 + r) for r in range(4)]
    eb = 1e-4
    s = oracle.compress(bufs[0], eb)
    exact = bufs[0].astype(np.float64)
    for k in range(1, 4):
        s = oracle.fused_step(s, bufs[k], eb)
        exact += bufs[k]
    e = oracle.decompress(s).astype(np.float64) - exact
    assert abs(e.mean()) < 0.05 * eb
    assert e.std() > 0.2 * eb  # the errors are really there


def test_scatter_chunks_are_single_streams(oracle):
    """Sec. 3.3.4 (gZ-Scatter): each chunk is its own complete stream, packed
    back to back; offsets are the exclusive sum of the sizes."""
    x = synth.sinusoids(50000, seed=12)
    counts, displs = synth.loguniform_counts(x.size, 7, 100, 20000, seed=3)
    packed, cb, co = oracle.scatter_compress(x, counts, displs, 1e-4, block_len=64)
    assert np.array_equal(co, np.concatenate([[0], np.cumsum(cb)[:-1]]))
    for j in range(len(counts)):
        d, c = int(displs[j]), int(counts[j])
        single = oracle.compress(x[d:d + c], 1e-4, block_len=64)
        assert packed[int(co[j]):int(co[j] + cb[j])].tobytes() == single.tobytes()


def test_mode1_exhaustive_is_min_of_trials(oracle):
    """Brute force: in exhaustive mode each tile takes the smallest of the
    three encodings (checked by re-encoding every tile with each predictor
    forced through a one-tile stream)."""
    g = np.random.default_rng(13)
    nx, ny = 32, 16
    fields = [np.cumsum(np.cumsum(g.normal(0, 1, (ny, nx)), 0), 1) * 0.05,
              g.normal(0, 1, (ny, nx)),
              np.outer(np.arange(ny), np.arange(nx)) * 0.01 + g.normal(0, 1e-3, (ny, nx))]
    eb = 1e-3
    t = np.float32(2 * eb)
    for f in fields:
        x = f.astype(np.float32).reshape(-1)
        s = oracle.compress(x, eb, block_len=64, mode=1, nx=nx, select=1)
        y = oracle.decompress(s)
        assert np.all(np.abs(y.astype(np.float64) - x) <= eb)
        hdr = s[64 + 4:64 + 4 + (nx // 8) * (ny // 8)]
        q = np.rint(y / t).astype(np.int32).reshape(ny, nx)
        kinds = {2: 0, 1: 1, 3: 2}
        for b in range(len(hdr)):
            R, C = divmod(b, nx // 8)
            tq = q[8 * R:8 * R + 8, 8 * C:8 * C + 8].reshape(64)
            sizes = oracle.tile_sizes(tq)
            kind = hdr[b] >> 5
            if kind in kinds:
                assert sizes[kinds[kind]] == sizes.min()
                assert kinds[kind] == int(np.argmin(sizes))  # first minimum


def test_tile_sizes_brute_force(oracle):
    """tile_sizes equals the payload length of a one-tile stream encoded with
    each predictor (NONE via a forced choice is not selectable, so NONE is
    checked against its definition: (F+1)*8 with F from max|q|)."""
    g = np.random.default_rng(14)
    for _ in range(50):
        q = g.integers(-300, 300, 64).astype(np.int32)
        s = oracle.tile_sizes(q)
        F = int(np.max(np.abs(q))).bit_length()
        assert s[0] == ((F + 1) * 8 if F else 0)
        x = q.astype(np.float32) * T13
        st = oracle.compress(x, EB14, block_len=64, mode=1, nx=8, select=2)
        pay = struct.unpack_from("<Q", st, 24)[0]
        assert pay == s[1] or (pay == 256 and s[1] > 256)


@pytest.mark.parametrize("corrupt", ["magic", "version", "truncated", "reserved_kind",
                                     "table", "payload_total", "pad", "zero_with_F",
                                     "none_in_mode0", "dtype", "log2L"])
def test_decoder_rejects_corruption(oracle, corrupt):
    x = synth.sinusoids(10000, seed=15)
    s = oracle.compress(x, 1e-4).copy()
    NS = -(-x.size // 4096)
    hoff = 64 + 4 * NS
    if corrupt == "magic":
        s[0] ^= 1
    elif corrupt == "version":
        s[4] = 2
    elif corrupt == "truncated":
        s = s[:-4]
    elif corrupt == "reserved_kind":
        s[hoff + 3] = (5 << 5)
    elif corrupt == "table":
        s[64 + 4] ^= 4
    elif corrupt == "payload_total":
        v = struct.unpack_from("<Q", s, 24)[0]
        s[24:32] = np.frombuffer(struct.pack("<Q", v - 4), np.uint8)
    elif corrupt == "pad":
        B = -(-x.size // 32)
        assert B % 4 != 0
        s[hoff + B] = 1
    elif corrupt == "zero_with_F":
        s[hoff + 1] = 0x03
    elif corrupt == "none_in_mode0":
        s[hoff + 1] = (2 << 5) | (s[hoff + 1] & 31)
    elif corrupt == "dtype":
        s[6] = 3
    elif corrupt == "log2L":
        s[7] = 4
    st, _ = oracle.decompress_status(s)
    assert st == oracle.ECORRUPT


def test_argument_errors(oracle):
    x = np.ones(100, np.float32)
    for eb in (0.0, -1.0, float("nan"), float("inf"), 1e-46):
        with pytest.raises(oracle.OracleError) as e:
            oracle.compress(x, eb)
        assert e.value.status == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, 1e-3, cap=100)
    assert e.value.status == oracle.ENOSPC
    with pytest.raises(oracle.OracleError):
        oracle.compress(x[:96], 1e-3, block_len=64, mode=1, nx=12, select=1)
    s = oracle.compress(x, 1e-3)
    st, _ = oracle.decompress_status(s, cap=50)
    assert st == oracle.ENOSPC


def test_subnormal_step_gives_raw(oracle):
    """A subnormal t is allowed; nearly everything fails the check and goes
    RAW, which still round-trips exactly."""
    x = np.linspace(-1, 1, 1000).astype(np.float32)
    s = oracle.compress(x, 1e-40)
    assert np.array_equal(oracle.decompress(s).view(np.uint32), x.view(np.uint32))


@pytest.mark.slow
def test_quantize_exhaustive_fp32(oracle):
    """All 2^32 float32 bit patterns against numpy's closed form."""
    for eb in (1e-4, 1e-3, 2.0 ** -14):
        t = np.float32(2 * eb)
        for hi in range(1 << 8):
            bits = (np.arange(1 << 24, dtype=np.uint64) + (hi << 24)).astype(np.uint32)
            x = bits.view(np.float32)
            q, fail = oracle.quantize(x, eb)
            with np.errstate(all="ignore"):
                r = x / t
                ok = np.isfinite(x) & (np.abs(r.astype(np.float64)) <= 536870911.0)
                qr = np.rint(np.where(ok, r, 0)).astype(np.int32)
                xh = qr.astype(np.float32) * t
                good = ok & (np.abs(x.astype(np.float64) - xh.astype(np.float64)) <= eb)
            assert np.array_equal(fail, ~good)
            assert np.array_equal(q[good], qr[good])


@pytest.mark.parametrize("L", [32, 64, 128])
def test_all_core_variants_write_the_same_bytes(oracle, L):
    """The OpenMP variants (superblocks at once, serial offset scan) give the
    scalar oracle's bytes and values: fp32 and fp64, a ragged tail, RAW and
    ZERO blocks, tile mode with every selector, and the fused step."""
    from paper_2308_05199_amd import synth
    rng = np.random.default_rng(L)
    n = 5 * 4096 + 1234
    x = synth.sinusoids(n, seed=L).astype(np.float64)
    x[100:4200] = 0.0
    x[7000] = np.nan
    x[9000:9100] = 1e12
    for dt in (np.float32, np.float64):
        xs = x.astype(dt)
        s = oracle.compress(xs, 1e-4, block_len=L)
        assert oracle.compress(xs, 1e-4, block_len=L, mt=True).tobytes() == s.tobytes()
        assert oracle.decompress(s, mt=True).tobytes() == oracle.decompress(s).tobytes()
    loc = rng.standard_normal(n).astype(np.float32)
    s = oracle.compress(x.astype(np.float32), 1e-4, block_len=L)
    assert (oracle.fused_step(s, loc, 1e-4, block_len=L, mt=True).tobytes() ==
            oracle.fused_step(s, loc, 1e-4, block_len=L).tobytes())
    if L == 64:
        t = synth.sinusoids(64 * 8 * 40, seed=3)
        blob = bytes(np.random.default_rng(0).integers(-3, 4, 756).astype(np.int8))
        blob = b"GZM1" + (4).to_bytes(4, "little") + blob[8:520] + bytes(4 * 32) + \
            blob[552:648] + bytes(12)
        for sel in (0, 1, 2):
            a = oracle.compress(t, 1e-4, block_len=64, mode=1, nx=64, select=sel, blob=blob)
            b = oracle.compress(t, 1e-4, block_len=64, mode=1, nx=64, select=sel, blob=blob,
                                mt=True)
            assert a.tobytes() == b.tobytes()
