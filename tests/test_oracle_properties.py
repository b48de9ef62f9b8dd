"""Property tests of the CPU oracle (random tiny arrays with NaN, +-Inf,
-0, subnormals, exact ties and huge values), checked against an independent
numpy statement of the quantiser and the block rules of the format:

* RAW exactly when an element fails the bound (non-finite, |r| >= 2^29 or
  |x - (T)q t| > eb) or the coded block would be larger than the raw one;
* ZERO exactly when every q is 0; otherwise L1D with the minimal width F;
* decoded values within eb (coded blocks) or bit-identical (RAW blocks);
* re-encoding the decoded values gives the same stream (idempotence).
"""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

SPECIALS = np.array([np.nan, np.inf, -np.inf, -0.0, 0.0, 1e-45, -1e-45, 1.1754942e-38,
                     3.0e38, -3.0e38, 65504.0], np.float32)


@st.composite
def cases(draw):
    eb = draw(st.sampled_from([2.0 ** -14, 1e-3, 1e-4, 0.37]))
    L = draw(st.sampled_from([32, 64, 128]))
    n = draw(st.integers(1, 300))
    t = np.float32(2 * eb)
    kinds = draw(st.lists(st.integers(0, 5), min_size=n, max_size=n))
    vals = draw(st.lists(st.integers(-2000, 2000), min_size=n, max_size=n))
    x = np.empty(n, np.float32)
    for i, (k, v) in enumerate(zip(kinds, vals)):
        if k == 0:
            x[i] = np.float32(v) * t                       # on the grid
        elif k == 1:
            x[i] = np.float32((v + 0.5) * np.float64(t))   # exact ties
        elif k == 2:
            x[i] = SPECIALS[abs(v) % SPECIALS.size]
        elif k == 3:
            x[i] = np.float32(v * 1e-3)                    # smooth-ish
        elif k == 4:
            x[i] = np.float32(v) * np.float32(1e4)         # large steps
        else:
            x[i] = x[i - 1] if i else np.float32(0)        # repeats
    return x, eb, L


def layout(n, L):
    NS = -(-n // 4096)
    B = -(-n // L)
    return 64 + 4 * NS, B


def quantise_np(x, eb):
    """The quantiser written independently in numpy: r = x / t in float32
    (IEEE), q = rint(r) (ties to even), fail when x is not finite,
    |r| >= 2^29 or |x - fl32(q t)| > eb."""
    t = np.float32(2 * eb)
    with np.errstate(all="ignore"):
        r = np.divide(x, t, dtype=np.float32)
        rr = np.rint(r)
        fin = np.isfinite(x) & (np.abs(r) < np.float32(2 ** 29))
        q = np.where(fin, rr, 0).astype(np.int64)
        xh = np.multiply(q.astype(np.float32), t, dtype=np.float32)
        err = np.abs(x.astype(np.float64) - xh.astype(np.float64))
    fail = ~fin | ~(err <= eb)
    return q, fail


@settings(max_examples=250, deadline=None)
@given(cases())
def test_block_rules_and_bound(oracle, case):
    x, eb, L = case
    n = x.size
    s = oracle.compress(x, eb, block_len=L)
    hoff, B = layout(n, L)
    heads = s[hoff:hoff + B]
    q, fail = quantise_np(x, eb)
    y = oracle.decompress(s)
    for b in range(B):
        lo, hi = b * L, min(n, (b + 1) * L)
        kind, F = int(heads[b]) >> 5, int(heads[b]) & 31
        qb = q[lo:hi]
        if fail[lo:hi].any():
            assert kind == 7, (b, "a failing element forces RAW")
        else:
            d = np.diff(qb, prepend=qb[0])  # d0 = 0: the base is stored whole
            need = int(np.abs(d).max()).bit_length()
            coded = 4 * (1 + ((need + 1) * (L // 32) if need else 0))  # base, sign, planes
            raw = 4 * (hi - lo)
            if not qb.any():
                assert kind == 0 and F == 0, b
            elif coded > raw:
                assert kind == 7, b
            else:
                assert kind == 1 and F == need, (b, F, need)
        if kind == 7:
            assert y[lo:hi].tobytes() == x[lo:hi].tobytes(), b
        else:
            assert np.all(np.abs(y[lo:hi].astype(np.float64) - x[lo:hi].astype(np.float64))
                          <= eb), b


@settings(max_examples=150, deadline=None)
@given(cases())
def test_reencoding_the_decoded_values_is_idempotent(oracle, case):
    x, eb, L = case
    s = oracle.compress(x, eb, block_len=L)
    assert oracle.compress(oracle.decompress(s), eb, block_len=L).tobytes() == s.tobytes()
