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
    "gz_ctx_status": ([_vp, ctypes.POINTER(_i32)], _i32),
    "gz_ctx_reset": ([_vp, _vp], _i32),
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
    "gz_tune": ([_vp, _i32, _u32, _u64, ctypes.c_char_p, _pp], _i32),
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


class GzError(RuntimeError):
    def __init__(self, status, what):
        msg = gz_status_str(status).decode()
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

    def device_status(self):
        st = _i32(0)
        check(gz_ctx_status(self.h, ctypes.byref(st)), "gz_ctx_status")
        return st.value

    def reset(self, stream=None):
        check(gz_ctx_reset(self.h, _stream(stream)), "gz_ctx_reset")

    def quantize(self, x, eb, stream=None):
        q = torch.empty(x.numel(), dtype=torch.int32, device=x.device)
        f = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
        check(gz_quantize(self.h, _ptr(x), x.numel(), _dt(x), eb, _ptr(q), _ptr(f),
                          _stream(stream)), "gz_quantize")
        return q, f

    def compress(self, x, eb, block_len=32, threads=0, grid=0, out=None, out_bytes=None,
                 stream=None):
        n = x.numel()
        cap = bound(n, _dt(x), block_len)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        if out_bytes is None:
            out_bytes = torch.zeros(1, dtype=torch.int64, device=x.device)
        p = _params(block_len, threads, grid)
        check(gz_compress(self.h, _ptr(x), n, _dt(x), eb, ctypes.byref(p), _ptr(out),
                          out.numel(), _ptr(out_bytes), _stream(stream)), "gz_compress")
        return out, out_bytes

    def decompress(self, stream_buf, n, dtype=torch.float32, block_len=32, in_bytes=None,
                   threads=0, grid=0, out=None, stream=None):
        if out is None:
            out = torch.empty(n, dtype=dtype, device=stream_buf.device)
        ib = stream_buf.numel() if in_bytes is None else in_bytes
        p = _params(block_len, threads, grid)
        check(gz_decompress(self.h, _ptr(stream_buf), ib, n, _dt(out), ctypes.byref(p),
                            _ptr(out), _stream(stream)), "gz_decompress")
        return out

    def fused_reduce_step(self, stream_in, local, eb, block_len=32, in_bytes=None, threads=0,
                          grid=0, out=None, out_bytes=None, stream=None):
        n = local.numel()
        cap = bound(n, GZ_F32, block_len)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=local.device)
        if out_bytes is None:
            out_bytes = torch.zeros(1, dtype=torch.int64, device=local.device)
        ib = stream_in.numel() if in_bytes is None else in_bytes
        p = _params(block_len, threads, grid)
        check(gz_fused_reduce_step(self.h, _ptr(stream_in), ib, _ptr(local), n, eb,
                                   ctypes.byref(p), _ptr(out), out.numel(), _ptr(out_bytes),
                                   _stream(stream)), "gz_fused_reduce_step")
        return out, out_bytes

    def decompress_add(self, stream_in, acc, block_len=32, in_bytes=None, threads=0, grid=0,
                       stream=None):
        """acc (fp32, on the device) += decoded stream, in place."""
        if acc.dtype != torch.float32 or not acc.is_contiguous() or not acc.is_cuda:
            raise GzError(GZ_EINVAL, "decompress_add: acc must be a contiguous fp32 device tensor")
        ib = stream_in.numel() if in_bytes is None else in_bytes
        p = _params(block_len, threads, grid)
        check(gz_decompress_add(self.h, _ptr(stream_in), ib, acc.numel(), ctypes.byref(p),
                                _ptr(acc), _stream(stream)), "gz_decompress_add")
        return acc

    def scatter_compress(self, root, counts, displs, eb, block_len=32, threads=0, grid=0,
                         out=None, stream=None):
        counts = np.ascontiguousarray(counts, dtype=np.uint64)
        displs = np.ascontiguousarray(displs, dtype=np.uint64)
        dt = _dt(root)
        cap = sum(bound(int(c), dt, block_len) for c in counts)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=root.device)
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
        total = int((displs + counts).max()) if len(counts) else 0
        if out is None:
            out = torch.empty(total, dtype=dtype, device=packed.device)
        pb = packed.numel() if packed_bytes is None else packed_bytes
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
            r.block_len = it.get("block_len", 32)
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
