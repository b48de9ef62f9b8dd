"""Exhaustive check of the GPU quantiser (opt-in: GZ_SLOW=1): every one of the
2^32 float32 bit patterns, in chunks of 2^28, through gz_quantize against an
independent numpy statement of the quantisation rule with numpy's IEEE
float32 division: r = x / t, FAIL if x is not finite or |r| > 2^29 - 1,
q = rint(r) (ties to even), FAIL unless |x - (float32)q * t| <= eb in
float64.  The kernel forms r as fl32((double)x * (1 / (double)t)) instead of
dividing; this sweep is what backs that replacement, for the bounds 1e-4,
1e-3, 2^-14 and the ring workload's 1e-4 x range."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CHUNK = 1 << 28


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def reference(xb, t, eb):
    """q (0 where FAIL) and FAIL for the float32 values with bits xb."""
    x = xb.view(np.float32)
    with np.errstate(all="ignore"):
        r = x / t
        fin = np.isfinite(x)
        inr = np.abs(r.astype(np.float64)) <= 536870911.0
        rr = np.rint(r)
        xh = rr.astype(np.float32) * t
        ok = fin & inr & (np.abs(x.astype(np.float64) - xh.astype(np.float64)) <= eb)
    q = np.where(ok, rr, 0).astype(np.int32)
    return q, ~ok


def check_chunk(xb, q, f, t, eb):
    parts = 16
    n = xb.size // parts

    def one(k):
        sl = slice(k * n, (k + 1) * n)
        rq, rf = reference(xb[sl], t, eb)
        return int(np.count_nonzero(rq != q[sl])), int(np.count_nonzero(rf != f[sl].astype(bool)))

    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(one, range(parts)))
    return sum(a for a, _ in res), sum(b for _, b in res)


@pytest.mark.parametrize("eb", [1e-4, 1e-3, 2.0 ** -14, 0.0010239075660705566])
def test_every_float32_bit_pattern(eb):
    import torch
    from paper_2308_05199_amd import gzccl as gz
    ctx = gz.Context(0, max_elems=1 << 20, max_requests=4)
    t = np.float32(2.0 * eb)
    bad_q = bad_f = 0
    for c in range(1 << 32 >> 28):
        lo = c * CHUNK                        # patterns lo .. lo + 2^28 - 1 as uint32
        start = lo if lo < (1 << 31) else lo - (1 << 32)   # the same bits as int32
        xd = torch.arange(start, start + CHUNK, dtype=torch.int32, device="cuda")
        xd = xd.view(torch.float32)
        q, f = ctx.quantize(xd, eb)
        torch.cuda.synchronize()
        xb = xd.view(torch.int32).cpu().numpy().view(np.uint32)
        assert int(xb[0]) == lo and int(xb[-1]) == lo + CHUNK - 1
        dq, df = check_chunk(xb, q.cpu().numpy(), f.cpu().numpy(), t, eb)
        bad_q += dq
        bad_f += df
        say(f"eb {eb:g} chunk {c}: q mismatches {dq}, FAIL mismatches {df}")
        del xd, q, f
    assert ctx.device_status() == 0
    ctx.close()
    assert bad_q == 0 and bad_f == 0
