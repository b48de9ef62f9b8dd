"""Python binding of the C ABI in include/gzccl.h.

Argument marshalling only: every step of the codec runs in the HIP kernels
of libgzccl.so.  PyTorch supplies device memory and streams.  The raw entry
points keep their C names (gz_compress, gz_decompress, ...); `Context` wraps
them for tensors.  There is no CPU fallback: without the built library this
module raises on import.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgzccl.so")

GZ_OK, GZ_EINVAL, GZ_ENOSPC, GZ_ECORRUPT, GZ_EHIP, GZ_ENOMEM, GZ_EUNSUPPORTED, GZ_ETIMEOUT = range(8)
GZ_F32, GZ_F64 = 0, 1
GZ_OP_COMPRESS, GZ_OP_DECOMPRESS, GZ_OP_FUSED, GZ_OP_ACCUMULATE = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2308_05199_amd/build.py "
                      "(the HIP library has no CPU fallback)")
lib = ctypes.CDLL(LIB_PATH)


class gz_params(ctypes.Structure):
    _fields_ = [("block_len", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("select", ctypes.c_uint32), ("nx", ctypes.c_uint32)]


class gz_request(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("local", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("d_out_bytes", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("in_bytes", ctypes.c_uint64), ("out_cap", ctypes.c_uint64),
                ("eb", ctypes.c_double), ("dtype", ctypes.c_uint32),
                ("block_len", ctypes.c_uint32)]


_vp, _u64, _u32, _i32, _dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
_pp = ctypes.POINTER(gz_params)
_SIGS = {
    "gz_ctx_create": ([ctypes.POINTER(_vp), _i32, _u64, _u32], _i32),
    "gz_ctx_destroy": ([_vp], None),
    "gz_ctx_status": ([_vp, _vp, ctypes.POINTER(_i32)], _i32),
    "gz_ctx_reset": ([_vp, _vp], _i32),
    "gz_ctx_set_wait": ([_vp, _u64], _i32),
    "gz_compress_bound": ([_u64, _i32, _u32], _u64),
    "gz_quantize": ([_vp, _vp, _u64, _i32, _dbl, _vp, _vp, _vp], _i32),
    "gz_compress": ([_vp, _vp, _u64, _i32, _dbl, _pp, _vp, _u64, _vp, _vp], _i32),
    "gz_decompress": ([_vp, _vp, _u64, _u64, _i32, _pp, _vp, _vp], _i32),
    "gz_fused_reduce_step": ([_vp, _vp, _u64, _vp, _u64, _dbl, _pp, _vp, _u64, _vp, _vp], _i32),
    "gz_decompress_add": ([_vp, _vp, _u64, _u64, _pp, _vp, _vp], _i32),
    "gz_scatter_compress": ([_vp, _vp, _i32, _vp, _vp, _u32, _dbl, _pp, _vp, _u64, _vp, _vp, _vp],
                            _i32),
    "gz_scatter_decompress": ([_vp, _vp, _u64, _vp, _i32, _vp, _vp, _u32, _pp, _vp, _vp], _i32),
    "gz_batch": ([_vp, _i32, ctypes.POINTER(gz_request), _u32, _pp, _vp], _i32),
    "gz_plan_create": ([_vp, _i32, ctypes.POINTER(gz_request), _u32, _pp, ctypes.POINTER(_vp)],
                       _i32),
    "gz_plan_launch": ([_vp, _vp], _i32),
    "gz_plan_destroy": ([_vp], None),
    "gz_graph_create": ([ctypes.POINTER(_vp), _u32, ctypes.POINTER(_vp)], _i32),
    "gz_graph_launch": ([_vp, _vp], _i32),
    "gz_graph_destroy": ([_vp], None),
    "gz_tune": ([_vp, _i32, _u32, _vp, _u64, _vp, _u64, ctypes.c_char_p, _pp, _vp], _i32),
    "gz_tune_batch": ([_vp, _i32, ctypes.POINTER(gz_request), _u32, ctypes.c_char_p, _pp, _vp],
                      _i32),
    "gz_selector_load": ([_vp, _vp, _u64], _i32),
    "gz_tile_trial": ([_vp, _vp, _u64, _u32, _dbl, _vp, _vp, _vp, _vp], _i32),
    "gz_mlp_grad": ([_vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp], _i32),
    "gz_mlp_adam": ([_vp, _vp, _vp, _vp, _vp, _u32, ctypes.c_float, _vp], _i32),
    "gz_compress_noalloc": ([_vp, _u64, _i32, _dbl, _pp, _vp, _u64, _vp, _vp, _vp], _i32),
    "gz_status_str": ([_i32], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f

EXPORTED = tuple(_SIGS)
_STATUS_TEXT = {k: gz_status_str(k).decode() for k in range(8)}


class GzError(RuntimeError):
    def __init__(self, status, what):
        msg = _STATUS_TEXT.get(status, "unknown status")
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


def check(status, what):
    if status != GZ_OK:
        raise GzError(status, what)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


_F = (torch.float32, torch.float64)


def _need(t, what, name, dtypes=None, numel=None):
    """Raises GzError (nothing is enqueued) unless t is a contiguous tensor on
    a GPU device, of one of `dtypes`, with at least `numel` elements: the C
    ABI takes raw device pointers, so a host tensor, a strided view or a
    narrower dtype would make the kernels read or write the wrong memory."""
    if not isinstance(t, torch.Tensor):
        raise GzError(GZ_EINVAL, f"{what}: {name} must be a torch tensor")
    if not t.is_contiguous():
        raise GzError(GZ_EINVAL, f"{what}: {name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise GzError(GZ_EINVAL, f"{what}: {name} must be {'/'.join(str(d) for d in dtypes)}, "
                                 f"not {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise GzError(GZ_EINVAL, f"{what}: {name} holds {t.numel()} elements, needs {numel}")
    if not _on_gpu(t):
        raise GzError(GZ_EINVAL, f"{what}: {name} must be on a GPU device, not {t.device}")
    return t


def _on_gpu(t):
    return t.is_cuda


def _dt(t):
    if t.dtype == torch.float32:
        return GZ_F32
    if t.dtype == torch.float64:
        return GZ_F64
    raise TypeError("float32 or float64 tensors only")


def _params(block_len=32, threads=0, grid=0, mode=0, select=0, nx=0):
    return gz_params(block_len, threads, grid, mode, select, nx)


def bound(n, dtype=GZ_F32, block_len=32):
    return int(gz_compress_bound(n, dtype, block_len))


def compress_noalloc(x, eb, out, out_bytes, status, block_len=32, threads=0, grid=0, mode=0,
                     select=0, nx=0, stream=None):
    """gz_compress without a context, for callers that cannot allocate:
    out (uint8, at least bound() bytes), out_bytes (int64[1]) and status
    (int32[1]) are caller-owned device tensors; nothing is allocated."""
    what = "gz_compress_noalloc"
    _need(x, what, "x", _F)
    _need(out, what, "out", (torch.uint8,), bound(x.numel(), _dt(x), block_len))
    _need(out_bytes, what, "out_bytes", (torch.int64,), 1)
    if status is not None:
        _need(status, what, "status", (torch.int32,), 1)
    p = _params(block_len, threads, grid, mode, select, nx)
    check(gz_compress_noalloc(_ptr(x), x.numel(), _dt(x), eb, ctypes.byref(p), _ptr(out),
                              out.numel(), _ptr(out_bytes), _ptr(status), _stream(stream)),
          "gz_compress_noalloc")
    return out, out_bytes


class Context:
    """A device workspace (tickets, look-back words, descriptor arena) sized
    once for calls of up to max_elems elements and max_requests requests."""

    def __init__(self, device=0, max_elems=1 << 28, max_requests=4096):
        self.device = device
        self.h = ctypes.c_void_p()
        check(gz_ctx_create(ctypes.byref(self.h), device, max_elems, max_requests),
              "gz_ctx_create")

    def close(self):
        if self.h:
            gz_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        """Clears the context's look-back and ticket state (after a device
        error such as an expired wait)."""
        check(gz_ctx_reset(self.h, _stream(stream)), "gz_ctx_reset")

    def set_wait(self, usec):
        """Bound of the kernels' waits between waves, in microseconds
        (default 1 s); an expired wait reports GZ_ETIMEOUT."""
        check(gz_ctx_set_wait(self.h, int(usec)), "gz_ctx_set_wait")

    def device_status(self, stream=None):
        """Waits for `stream` (default: the current one) and returns and
        clears the sticky device status."""
        st = _i32(0)
        check(gz_ctx_status(self.h, _stream(stream), ctypes.byref(st)), "gz_ctx_status")
        return st.value

    def tune(self, sample, block_len=0, cache_path=None, stream=None):
        """Autotunes launch shapes (and, with block_len 0, the block length of
        requests that give 0) for single calls of sample's dtype and size,
        timed on the sample itself.  Returns the best params."""
        what = "gz_tune"
        _need(sample, what, "sample", _F)
        n = sample.numel()
        es = sample.element_size()
        r256 = lambda a: (a + 255) // 256 * 256
        work = torch.empty(r256(n * es) + r256(bound(n, _dt(sample), 32)) + 8,
                           dtype=torch.uint8, device=sample.device)
        best = gz_params()
        cp = cache_path.encode() if isinstance(cache_path, str) else cache_path
        check(gz_tune(self.h, _dt(sample), block_len, _ptr(sample), n, _ptr(work),
                      work.numel(), cp, ctypes.byref(best), _stream(stream)), what)
        return best

    def tune_batch(self, op, reqs, cache_path=None, stream=None):
        """Autotunes (threads, grid) of this batch's op and element-type mix;
        runs the batch in place.  Returns the best params."""
        best = gz_params()
        cp = cache_path.encode() if isinstance(cache_path, str) else cache_path
        check(gz_tune_batch(self.h, op, reqs, len(reqs), cp, ctypes.byref(best),
                            _stream(stream)), "gz_tune_batch")
        return best

    def quantize(self, x, eb, stream=None):
        _need(x, "gz_quantize", "x", _F)
        q = torch.empty(x.numel(), dtype=torch.int32, device=x.device)
        f = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
        check(gz_quantize(self.h, _ptr(x), x.numel(), _dt(x), eb, _ptr(q), _ptr(f),
                          _stream(stream)), "gz_quantize")
        return q, f

    def compress(self, x, eb, block_len=32, threads=0, grid=0, out=None, out_bytes=None,
                 stream=None):
        what = "gz_compress"
        _need(x, what, "x", _F)
        n = x.numel()
        cap = bound(n, _dt(x), block_len)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        if out_bytes is None:
            out_bytes = torch.zeros(1, dtype=torch.int64, device=x.device)
        _need(out, what, "out", (torch.uint8,))
        _need(out_bytes, what, "out_bytes", (torch.int64,), 1)
        p = _params(block_len, threads, grid)
        check(gz_compress(self.h, _ptr(x), n, _dt(x), eb, ctypes.byref(p), _ptr(out),
                          out.numel(), _ptr(out_bytes), _stream(stream)), "gz_compress")
        return out, out_bytes

    def decompress(self, stream_buf, n, dtype=torch.float32, block_len=32, in_bytes=None,
                   threads=0, grid=0, out=None, stream=None):
        what = "gz_decompress"
        _need(stream_buf, what, "stream_buf", (torch.uint8,))
        if out is None:
            out = torch.empty(n, dtype=dtype, device=stream_buf.device)
        _need(out, what, "out", _F, n)
        ib = stream_buf.numel() if in_bytes is None else in_bytes
        if ib > stream_buf.numel():
            raise GzError(GZ_EINVAL, f"{what}: in_bytes {ib} exceeds the buffer")
        p = _params(block_len, threads, grid)
        check(gz_decompress(self.h, _ptr(stream_buf), ib, n, _dt(out), ctypes.byref(p),
                            _ptr(out), _stream(stream)), "gz_decompress")
        return out

    def fused_reduce_step(self, stream_in, local, eb, block_len=32, in_bytes=None, threads=0,
                          grid=0, out=None, out_bytes=None, stream=None):
        what = "gz_fused_reduce_step"
        _need(stream_in, what, "stream_in", (torch.uint8,))
        _need(local, what, "local", (torch.float32,))
        n = local.numel()
        cap = bound(n, GZ_F32, block_len)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=local.device)
        if out_bytes is None:
            out_bytes = torch.zeros(1, dtype=torch.int64, device=local.device)
        _need(out, what, "out", (torch.uint8,))
        _need(out_bytes, what, "out_bytes", (torch.int64,), 1)
        ib = stream_in.numel() if in_bytes is None else in_bytes
        if ib > stream_in.numel():
            raise GzError(GZ_EINVAL, f"{what}: in_bytes {ib} exceeds the buffer")
        p = _params(block_len, threads, grid)
        check(gz_fused_reduce_step(self.h, _ptr(stream_in), ib, _ptr(local), n, eb,
                                   ctypes.byref(p), _ptr(out), out.numel(), _ptr(out_bytes),
                                   _stream(stream)), "gz_fused_reduce_step")
        return out, out_bytes

    def decompress_add(self, stream_in, acc, block_len=32, in_bytes=None, threads=0, grid=0,
                       stream=None):
        """acc (fp32, on the device) += decoded stream, in place."""
        what = "gz_decompress_add"
        _need(stream_in, what, "stream_in", (torch.uint8,))
        _need(acc, what, "acc", (torch.float32,))
        ib = stream_in.numel() if in_bytes is None else in_bytes
        if ib > stream_in.numel():
            raise GzError(GZ_EINVAL, f"{what}: in_bytes {ib} exceeds the buffer")
        p = _params(block_len, threads, grid)
        check(gz_decompress_add(self.h, _ptr(stream_in), ib, acc.numel(), ctypes.byref(p),
                                _ptr(acc), _stream(stream)), "gz_decompress_add")
        return acc

    def scatter_compress(self, root, counts, displs, eb, block_len=32, threads=0, grid=0,
                         out=None, stream=None):
        what = "gz_scatter_compress"
        counts = np.ascontiguousarray(counts, dtype=np.uint64)
        displs = np.ascontiguousarray(displs, dtype=np.uint64)
        _need(root, what, "root", _F, int((displs + counts).max()) if len(counts) else 0)
        dt = _dt(root)
        cap = sum(bound(int(c), dt, block_len) for c in counts)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=root.device)
        _need(out, what, "out", (torch.uint8,))
        cb = torch.zeros(len(counts), dtype=torch.int64, device=root.device)
        co = torch.zeros(len(counts), dtype=torch.int64, device=root.device)
        p = _params(block_len, threads, grid)
        check(gz_scatter_compress(self.h, _ptr(root), dt,
                                  counts.ctypes.data_as(_vp), displs.ctypes.data_as(_vp),
                                  len(counts), eb, ctypes.byref(p), _ptr(out), out.numel(),
                                  _ptr(cb), _ptr(co), _stream(stream)), "gz_scatter_compress")
        return out, cb, co

    def scatter_decompress(self, packed, chunk_offsets, counts, displs, dtype=torch.float32,
                           block_len=32, packed_bytes=None, threads=0, grid=0, out=None,
                           stream=None):
        counts = np.ascontiguousarray(counts, dtype=np.uint64)
        displs = np.ascontiguousarray(displs, dtype=np.uint64)
        what = "gz_scatter_decompress"
        total = int((displs + counts).max()) if len(counts) else 0
        _need(packed, what, "packed", (torch.uint8,))
        _need(chunk_offsets, what, "chunk_offsets", (torch.int64,), len(counts))
        if out is None:
            out = torch.empty(total, dtype=dtype, device=packed.device)
        _need(out, what, "out", _F, total)
        pb = packed.numel() if packed_bytes is None else packed_bytes
        if pb > packed.numel():
            raise GzError(GZ_EINVAL, f"{what}: packed_bytes {pb} exceeds the buffer")
        p = _params(block_len, threads, grid)
        check(gz_scatter_decompress(self.h, _ptr(packed), pb, _ptr(chunk_offsets), _dt(out),
                                    counts.ctypes.data_as(_vp), displs.ctypes.data_as(_vp),
                                    len(counts), ctypes.byref(p), _ptr(out), _stream(stream)),
              "gz_scatter_decompress")
        return out

    @staticmethod
    def requests(items):
        """items: dicts with in/local/out/out_bytes tensors and n, in_bytes,
        out_cap, eb, dtype, block_len.  Returns a ctypes array (keep the
        tensors alive while it is in use)."""
        arr = (gz_request * len(items))()
        for i, it in enumerate(items):
            what = f"request {i}"
            n = int(it["n"])
            es = 4 if it["dtype"] == GZ_F32 else 8
            for key in ("in", "out"):
                t = it.get(key)
                if t is None:
                    continue
                _need(t, what, key, (torch.uint8,) + _F)
                if t.dtype == torch.uint8:   # a stream: its stated size must fit
                    need = it.get("in_bytes", 0) if key == "in" else it.get("out_cap", 0)
                    if t.numel() < need:
                        raise GzError(GZ_EINVAL, f"{what}: {key} holds {t.numel()} bytes, "
                                                 f"needs {need}")
                elif t.numel() * t.element_size() < n * es:
                    raise GzError(GZ_EINVAL, f"{what}: {key} holds fewer than {n} elements")
            if it.get("local") is not None:
                _need(it["local"], what, "local", (torch.float32,), n)
            if it.get("out_bytes") is not None:
                _need(it["out_bytes"], what, "out_bytes", (torch.int64,), 1)
            r = arr[i]
            r.in_ = it["in"].data_ptr() if it.get("in") is not None else 0
            r.local = it["local"].data_ptr() if it.get("local") is not None else 0
            r.out = it["out"].data_ptr() if it.get("out") is not None else 0
            r.d_out_bytes = it["out_bytes"].data_ptr() if it.get("out_bytes") is not None else 0
            r.n = it["n"]
            r.in_bytes = it.get("in_bytes", 0)
            r.out_cap = it.get("out_cap", 0)
            r.eb = it.get("eb", 0.0)
            r.dtype = it["dtype"]
            r.block_len = it.get("block_len", 32)   # 0: the tuned length
        return arr

    def batch(self, op, reqs, threads=0, grid=0, stream=None):
        p = _params(32, threads, grid)
        check(gz_batch(self.h, op, reqs, len(reqs), ctypes.byref(p), _stream(stream)), "gz_batch")

    def plan(self, op, reqs, threads=0, grid=0):
        p = _params(32, threads, grid)
        h = ctypes.c_void_p()
        check(gz_plan_create(self.h, op, reqs, len(reqs), ctypes.byref(p), ctypes.byref(h)),
              "gz_plan_create")
        return Plan(h, reqs)


class Plan:
    def __init__(self, h, reqs):
        self.h, self._reqs = h, reqs

    def launch(self, stream=None):
        check(gz_plan_launch(self.h, _stream(stream)), "gz_plan_launch")

    def close(self):
        if self.h:
            gz_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """One HIP graph replaying a sequence of plans."""

    def __init__(self, plans):
        arr = (_vp * len(plans))(*[p.h.value for p in plans])
        self.h = ctypes.c_void_p()
        self._plans = plans
        check(gz_graph_create(arr, len(plans), ctypes.byref(self.h)), "gz_graph_create")

    def launch(self, stream=None):
        check(gz_graph_launch(self.h, _stream(stream)), "gz_graph_launch")

    def close(self):
        if self.h:
            gz_graph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
