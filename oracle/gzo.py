"""ctypes wrapper of the plain-C oracle (gzo.c).  Test infrastructure only."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOSPC, ECORRUPT = 0, 1, 2, 3
F32, F64 = 0, 1


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def build(force=True):
    """Compile gzo.c into liboracle.so (IEEE arithmetic, no contraction)."""
    src = os.path.join(_HERE, "gzo.c")
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64, i32, u32, dbl, vp = (ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                  ctypes.c_double, ctypes.c_void_p)
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        L.gzo_compress_bound.restype = u64
        L.gzo_compress_bound.argtypes = [u64, i32, i32]
        L.gzo_quantize.argtypes = [vp, u64, i32, dbl, vp, vp]
        L.gzo_compress.argtypes = [vp, u64, i32, dbl, i32, i32, u32, i32, vp, vp,
                                   u64, pu64]
        L.gzo_stream_info.argtypes = [vp, u64, pu64, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(u32), ctypes.POINTER(dbl), pu64]
        L.gzo_decompress.argtypes = [vp, u64, vp, u64, pu64]
        L.gzo_fused_step.argtypes = [vp, u64, vp, u64, dbl, i32, vp, u64, pu64]
        L.gzo_scatter_compress.argtypes = [vp, i32, vp, vp, u32, dbl, i32, vp, u64,
                                           vp, vp]
        L.gzo_tile_features.argtypes = [vp, vp]
        L.gzo_tile_features.restype = None
        L.gzo_mlp_forward.argtypes = [vp, vp, vp]
        L.gzo_mlp_blob_bytes.restype = u64
        L.gzo_tile_sizes.argtypes = [vp, vp]
        L.gzo_tile_sizes.restype = None
        L.gzo_tile_trial.argtypes = [vp, u64, u32, dbl, vp, vp, vp]
        L.gzo_threads.restype = i32
        L.gzo_compress_mt.argtypes = L.gzo_compress.argtypes
        L.gzo_decompress_mt.argtypes = L.gzo_decompress.argtypes
        L.gzo_fused_step_mt.argtypes = L.gzo_fused_step.argtypes
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(x):
    if x.dtype == np.float32:
        return F32
    if x.dtype == np.float64:
        return F64
    raise TypeError("oracle takes float32 or float64 arrays")


def compress_bound(n, dtype=F32, block_len=32):
    return int(lib().gzo_compress_bound(n, dtype, block_len))


def quantize(x, eb):
    x = np.ascontiguousarray(x)
    q = np.zeros(x.size, np.int32)
    f = np.zeros(x.size, np.uint8)
    st = lib().gzo_quantize(_ptr(x), x.size, _dtype_code(x), eb, _ptr(q), _ptr(f))
    if st:
        raise OracleError(st, "quantize")
    return q, f.astype(bool)


def threads():
    """Host threads the all-core (mt=True) variants use."""
    return int(lib().gzo_threads())


def compress(x, eb, block_len=32, mode=0, nx=0, select=0, blob=None, cap=None, mt=False):
    """Returns the GZ1 stream of x as a uint8 array (mt: on all host cores,
    same bytes)."""
    x = np.ascontiguousarray(x)
    dt = _dtype_code(x)
    need = compress_bound(x.size, dt, block_len)
    out = np.zeros(need if cap is None else cap, np.uint8)
    nb = ctypes.c_uint64(0)
    b = None
    if blob is not None:
        b = np.frombuffer(bytes(blob), np.uint8).copy()
    fn = lib().gzo_compress_mt if mt else lib().gzo_compress
    st = fn(_ptr(x), x.size, dt, eb, block_len, mode, nx, select,
            _ptr(b) if b is not None else None, _ptr(out), out.size, ctypes.byref(nb))
    if st:
        raise OracleError(st, "compress")
    return out[:nb.value].copy()


def stream_info(s):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    n = ctypes.c_uint64()
    dt, L, mode = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    nx = ctypes.c_uint32()
    eb = ctypes.c_double()
    tot = ctypes.c_uint64()
    st = lib().gzo_stream_info(_ptr(s), s.size, ctypes.byref(n), ctypes.byref(dt),
                               ctypes.byref(L), ctypes.byref(mode), ctypes.byref(nx),
                               ctypes.byref(eb), ctypes.byref(tot))
    if st:
        raise OracleError(st, "stream_info")
    return dict(n=n.value, dtype=dt.value, block_len=L.value, mode=mode.value,
                nx=nx.value, eb=eb.value, total_bytes=tot.value)


def decompress_status(s, cap=None, mt=False):
    """(status, array) without raising."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    try:
        info = stream_info(s)
    except OracleError as e:
        return e.status, None
    n = info["n"] if cap is None else cap
    out = np.zeros(max(n, 1), np.float32 if info["dtype"] == F32 else np.float64)
    got = ctypes.c_uint64()
    fn = lib().gzo_decompress_mt if mt else lib().gzo_decompress
    st = fn(_ptr(s), s.size, _ptr(out), n, ctypes.byref(got))
    if st:
        return st, None
    return OK, out[:got.value]


def decompress(s, mt=False):
    st, out = decompress_status(s, mt=mt)
    if st:
        raise OracleError(st, "decompress")
    return out


def fused_step(stream, local, eb, block_len=32, mt=False):
    local = np.ascontiguousarray(local, dtype=np.float32)
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.zeros(compress_bound(local.size, F32, block_len), np.uint8)
    nb = ctypes.c_uint64(0)
    fn = lib().gzo_fused_step_mt if mt else lib().gzo_fused_step
    st = fn(_ptr(stream), stream.size, _ptr(local), local.size, eb, block_len, _ptr(out),
            out.size, ctypes.byref(nb))
    if st:
        raise OracleError(st, "fused_step")
    return out[:nb.value].copy()


def scatter_compress(root, counts, displs, eb, block_len=32):
    root = np.ascontiguousarray(root)
    dt = _dtype_code(root)
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    displs = np.ascontiguousarray(displs, dtype=np.uint64)
    cap = sum(compress_bound(int(c), dt, block_len) for c in counts)
    out = np.zeros(max(cap, 1), np.uint8)
    cb = np.zeros(len(counts), np.uint64)
    co = np.zeros(len(counts), np.uint64)
    st = lib().gzo_scatter_compress(_ptr(root), dt, _ptr(counts), _ptr(displs),
                                    len(counts), eb, block_len, _ptr(out), out.size,
                                    _ptr(cb), _ptr(co))
    if st:
        raise OracleError(st, "scatter_compress")
    total = int(co[-1] + cb[-1]) if len(counts) else 0
    return out[:total].copy(), cb, co


def tile_features(qtile):
    q = np.ascontiguousarray(qtile, dtype=np.int32).reshape(64)
    f = np.zeros(16, np.int8)
    lib().gzo_tile_features(_ptr(q), _ptr(f))
    return f


def mlp_forward(blob, feat):
    b = np.frombuffer(bytes(blob), np.uint8).copy()
    f = np.ascontiguousarray(feat, dtype=np.int8)
    logits = np.zeros(3, np.int32)
    k = lib().gzo_mlp_forward(_ptr(b), _ptr(f), _ptr(logits))
    if k < 0:
        raise OracleError(EINVAL, "mlp_forward (bad blob)")
    return k, logits


def mlp_blob_bytes():
    return int(lib().gzo_mlp_blob_bytes())


def tile_sizes(qtile):
    q = np.ascontiguousarray(qtile, dtype=np.int32).reshape(64)
    s = np.zeros(3, np.uint32)
    lib().gzo_tile_sizes(_ptr(q), _ptr(s))
    return s


def tile_trial(x, nx, eb):
    """(features int8[B,16], sizes uint32[B,3], labels uint8[B]) per tile."""
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    B = x.size // 64
    f = np.zeros((B, 16), np.int8)
    s = np.zeros((B, 3), np.uint32)
    lab = np.zeros(B, np.uint8)
    st = lib().gzo_tile_trial(_ptr(x), x.size, nx, eb, _ptr(f), _ptr(s), _ptr(lab))
    if st:
        raise OracleError(st, "tile_trial")
    return f, s, lab
