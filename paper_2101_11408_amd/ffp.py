"""ctypes binding of libffp.so (include/ffp.h).

Argument marshalling only: every step of parsing runs in the HIP kernels of
the library.  PyTorch provides device memory and streams.  If the library has
not been built, importing the binding raises -- there is no CPU fallback.
"""

import atexit
import ctypes
import os
import sys
import weakref

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libffp.so")

# ffp_token_status
FFP_OK = 0
FFP_INVALID = 1
FFP_OUT_OF_RANGE = 2

# ffp_error
FFP_SUCCESS = 0
FFP_E_ARG = -1
FFP_E_CAPACITY = -2
FFP_E_HIP = -3
FFP_E_NOMEM = -4
FFP_E_BUDGET = -5
FFP_E_BUSY = -6
FFP_E_QUEUE = -7
FFP_E_INTERNAL = -8
FFP_E_SIZE = -9
NOALLOC_MAX_BYTES = 8 << 20

FFP_REJECT_PLUS = 1
FFP_JSON = 2
FFP_INFNAN = 4
FFP_HEX = 8
FFP_JSON_DOCUMENT = 0x40
FFP_CSV = 0x80
FFP_ROUND_MASK = 0x30
FFP_ROUND_NEAREST = 0x00
FFP_ROUND_TOWARD_ZERO = 0x10
FFP_ROUND_UP = 0x20
FFP_ROUND_DOWN = 0x30

DTYPE_F64 = 0
DTYPE_F32 = 1
DTYPE_F16 = 2
DTYPE_BF16 = 3

FFP_SERVE_BATCHED = 0
FFP_SERVE_PLAIN = 1


class ffp_options(ctypes.Structure):
    _fields_ = [("delim_set", ctypes.c_uint64 * 4), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ffp_job(ctypes.Structure):
    _fields_ = [("text", ctypes.c_void_p), ("nbytes", ctypes.c_uint64),
                ("values", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("dtype", ctypes.c_int32), ("err", ctypes.c_int32)]


class ffp_tuning(ctypes.Structure):
    _fields_ = [("tile_k", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("block_kib", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ffp_server_options(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("max_batch_jobs", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("spin_us", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class ffp_result(ctypes.Structure):
    _fields_ = [("values", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("count", ctypes.c_uint64), ("nbytes", ctypes.c_uint64),
                ("dtype", ctypes.c_int32), ("err", ctypes.c_int32),
                ("t_arrive_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("batch_jobs", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ffp_replay_request(ctypes.Structure):
    _fields_ = [("text", ctypes.c_void_p), ("nbytes", ctypes.c_uint64),
                ("on_device", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("arrival_ns", ctypes.c_uint64), ("dst_values", ctypes.c_void_p),
                ("dst_status", ctypes.c_void_p), ("dst_capacity", ctypes.c_uint64)]


class ffp_replay_result(ctypes.Structure):
    _fields_ = [("t_arrive_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("err", ctypes.c_int32), ("batch_jobs", ctypes.c_uint32)]


class ffp_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("submitted", "completed", "batches", "bytes", "arena_bytes",
                 "arena_peak_bytes", "scratch_bytes", "max_batch_seen", "cancelled")]


_c = ctypes
_P = _c.c_void_p
_U64 = _c.c_uint64
_I64 = _c.c_int64
_INT = _c.c_int

# name -> (restype, argtypes)
_SIGNATURES = {
    "ffp_create": (_INT, [_INT, _c.POINTER(ffp_options), _c.POINTER(_P)]),
    "ffp_destroy": (None, [_P]),
    "ffp_strerror": (_c.c_char_p, [_INT]),
    "ffp_reserve": (_INT, [_P, _U64]),
    "ffp_parse_f64": (_INT, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f64_noalloc": (_INT, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f32": (_INT, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f64_sync": (_I64, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f32_sync": (_I64, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f16": (_INT, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_bf16": (_INT, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_f16_sync": (_I64, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_parse_bf16_sync": (_I64, [_P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ffp_last_device_error": (_INT, [_P]),
    "ffp_timing_enable": (_INT, [_P, _INT]),
    "ffp_timing_read": (_INT, [_P, _c.POINTER(_c.c_double), _c.POINTER(_U64)]),
    "ffp_counters_enable": (_INT, [_P, _INT]),
    "ffp_set_reduce": (_INT, [_P, _P]),
    "ffp_set_reduce_sum": (_INT, [_P, _P]),
    "ffp_set_csv_columns": (_INT, [_P, _U64]),
    "ffp_counters_read": (_INT, [_P, _U64 * 6]),
    "ffp_parse_batch": (_INT, [_P, _P, _c.c_uint32, _U64, _P]),
    "ffp_batch_graph_create": (_INT, [_P, _P, _c.c_uint32, _U64, _c.POINTER(_P)]),
    "ffp_batch_graph_launch": (_INT, [_P, _P]),
    "ffp_batch_graph_destroy": (None, [_P]),
    "ffp_get_tuning": (_INT, [_P, _c.POINTER(ffp_tuning)]),
    "ffp_set_tuning": (_INT, [_P, _c.POINTER(ffp_tuning)]),
    "ffp_autotune_batch": (_INT, [_P, _P, _c.c_uint32, _U64, _P, _c.POINTER(ffp_tuning)]),
    "ffp_clock_ns": (_U64, []),
    "ffp_server_create": (_INT, [_P, _c.POINTER(ffp_server_options), _c.POINTER(_P)]),
    "ffp_server_submit": (_INT, [_P, _P, _U64, _INT, _INT, _U64, _c.POINTER(_U64)]),
    "ffp_server_poll": (_INT, [_P, _U64, _c.POINTER(ffp_result)]),
    "ffp_server_wait": (_INT, [_P, _U64, _c.POINTER(ffp_result)]),
    "ffp_server_copy_result": (_INT, [_P, _U64, _P, _P, _U64, _P]),
    "ffp_server_release": (_INT, [_P, _U64]),
    "ffp_server_stats_read": (_INT, [_P, _c.POINTER(ffp_server_stats)]),
    "ffp_server_destroy": (None, [_P]),
    "ffp_server_replay": (_INT, [_P, _P, _U64, _P]),
}

_lib = None

# Live handles, closed by an exit hook before the interpreter tears down its
# modules: a finalizer that ran during that teardown (or after the HIP
# runtime's own exit handlers) would call into HIP too late.  Servers are
# closed first, then graphs, then the contexts they were made from.
_live = {"server": weakref.WeakSet(), "graph": weakref.WeakSet(), "ctx": weakref.WeakSet()}


def _close_all():
    for kind in ("server", "graph", "ctx"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(_close_all)


def _finalize(obj):
    """__del__ body: close unless the interpreter is already shutting down
    (the exit hook has closed every live handle by then)."""
    if sys.is_finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


def load(path: str = LIB_PATH):
    """Load libffp.so (once) and declare the C-ABI prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            "libffp.so is not built (%s); run `python -m paper_2101_11408_amd.build` "
            "or __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


class FFPError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        lib = load()
        msg = lib.ffp_strerror(code).decode()
        super().__init__("%s%s (%d)" % (what + ": " if what else "", msg, code))
        self.code = code


def check(code: int, what: str = "") -> int:
    if code < 0:
        raise FFPError(code, what)
    return code


def make_options(delims: bytes = b"\n", flags: int = 0) -> ffp_options:
    o = ffp_options()
    for c in set(delims):
        o.delim_set[c >> 6] |= 1 << (c & 63)
    o.flags = flags
    return o


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def ffp_create(device: int = 0, delims: bytes = b"\n", flags: int = 0):
    lib = load()
    out = _P()
    opts = make_options(delims, flags)
    check(lib.ffp_create(device, ctypes.byref(opts), ctypes.byref(out)), "ffp_create")
    return out


def ffp_destroy(ctx):
    load().ffp_destroy(ctx)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def ffp_parse_f64(ctx, text, nbytes, values, status, capacity, count, stream=None):
    return load().ffp_parse_f64(ctx, text, nbytes, values, status, capacity, count,
                                _stream_handle(stream))


def ffp_parse_f32(ctx, text, nbytes, values, status, capacity, count, stream=None):
    return load().ffp_parse_f32(ctx, text, nbytes, values, status, capacity, count,
                                _stream_handle(stream))


def ffp_parse_f64_sync(ctx, text, nbytes, values, status, capacity, count, stream=None):
    return load().ffp_parse_f64_sync(ctx, text, nbytes, values, status, capacity, count,
                                     _stream_handle(stream))


def ffp_parse_f32_sync(ctx, text, nbytes, values, status, capacity, count, stream=None):
    return load().ffp_parse_f32_sync(ctx, text, nbytes, values, status, capacity, count,
                                     _stream_handle(stream))


# ---------------------------------------------------------------------------
# torch convenience layer (memory management only)
# ---------------------------------------------------------------------------

class Context:
    """Owns an ffp_ctx on one device."""

    def __init__(self, device: int = 0, delims: bytes = b"\n", flags: int = 0):
        self.device = device
        self.handle = ffp_create(device, delims, flags)
        _live["ctx"].add(self)

    def close(self):
        if self.handle:
            ffp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _finalize is not None:  # None once the module is torn down
            _finalize(self)

    def reserve(self, nbytes: int):
        check(load().ffp_reserve(self.handle, nbytes), "ffp_reserve")

    def timing(self, enable: bool = True):
        check(load().ffp_timing_enable(self.handle, 1 if enable else 0))

    def timing_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        check(load().ffp_timing_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def counters(self, enable: bool = True):
        check(load().ffp_counters_enable(self.handle, 1 if enable else 0))

    def set_reduce(self, out=None):
        """out: device int64 tensor of 3 elements (min bits, max bits, count)
        written by every later plain call; None turns the reduction off."""
        check(load().ffp_set_reduce(self.handle, out.data_ptr() if out is not None else None))

    def set_csv_columns(self, columns: int):
        """FFP_CSV contexts: bit c of `columns` selects column c."""
        check(load().ffp_set_csv_columns(self.handle, columns & 0xFFFFFFFFFFFFFFFF))

    def set_reduce_sum(self, out=None):
        """out: device int64 tensor of 2 elements (binary64 bits of the exact
        sum rounded once, 1 if exact) written by every later plain call;
        None turns the sum off."""
        check(load().ffp_set_reduce_sum(self.handle,
                                        out.data_ptr() if out is not None else None))

    def counters_read(self):
        arr = (ctypes.c_uint64 * 6)()
        check(load().ffp_counters_read(self.handle, arr))
        keys = ["tokens", "invalid", "early", "one", "two", "fallback"]
        return dict(zip(keys, list(arr)))

    def last_device_error(self) -> int:
        return load().ffp_last_device_error(self.handle)

    def parse_into(self, text, values, status, count, nbytes=None, stream=None,
                   sync=False):
        """Parse device uint8 tensor `text` into preallocated device tensors;
        the values tensor's dtype (float64, float32, float16, bfloat16) picks
        the output format."""
        import torch
        assert text.is_cuda and text.dtype == torch.uint8 and text.is_contiguous()
        name = {torch.float64: "f64", torch.float32: "f32", torch.float16: "f16",
                torch.bfloat16: "bf16"}[values.dtype]
        nb = text.numel() if nbytes is None else nbytes
        cap = min(values.numel(), status.numel())
        lib = load()
        fn = getattr(lib, "ffp_parse_%s%s" % (name, "_sync" if sync else ""))
        rc = fn(self.handle, text.data_ptr(), nb, values.data_ptr(), status.data_ptr(), cap,
                count.data_ptr(), _stream_handle(stream))
        return rc if sync else check(rc, "parse")

    def parse_into_noalloc(self, text, values, status, count, nbytes=None, stream=None):
        """ffp_parse_f64_noalloc into preallocated binary64 outputs: the call
        that allocates nothing (texts of up to NOALLOC_MAX_BYTES)."""
        import torch
        assert text.is_cuda and text.dtype == torch.uint8 and text.is_contiguous()
        assert values.dtype == torch.float64
        nb = text.numel() if nbytes is None else nbytes
        cap = min(values.numel(), status.numel())
        return check(load().ffp_parse_f64_noalloc(self.handle, text.data_ptr(), nb,
                                                  values.data_ptr(), status.data_ptr(), cap,
                                                  count.data_ptr(), _stream_handle(stream)),
                     "ffp_parse_f64_noalloc")

    # -- batched calls -------------------------------------------------
    def parse_batch(self, d_jobs, njobs, max_total_bytes, stream=None):
        """d_jobs: device tensor holding njobs ffp_job records (JobTable.dev)."""
        return check(load().ffp_parse_batch(self.handle, d_jobs.data_ptr(), njobs,
                                            max_total_bytes, _stream_handle(stream)),
                     "ffp_parse_batch")

    def get_tuning(self):
        t = ffp_tuning()
        check(load().ffp_get_tuning(self.handle, ctypes.byref(t)))
        return t.tile_k, t.blocks_per_cu

    def set_tuning(self, tile_k, blocks_per_cu=0, block_kib=0):
        t = ffp_tuning(tile_k, blocks_per_cu, block_kib)
        check(load().ffp_set_tuning(self.handle, ctypes.byref(t)), "ffp_set_tuning")

    def autotune_batch(self, d_jobs, njobs, max_total_bytes, stream=None):
        t = ffp_tuning()
        check(load().ffp_autotune_batch(self.handle, d_jobs.data_ptr(), njobs, max_total_bytes,
                                        _stream_handle(stream), ctypes.byref(t)),
              "ffp_autotune_batch")
        return t.tile_k, t.blocks_per_cu

    def parse(self, text, dtype=None, capacity=None, stream=None):
        """Parse a device uint8 tensor; returns (values, status) of the exact
        token count (a second pass with a larger capacity if needed)."""
        import torch
        dtype = dtype or torch.float64
        if capacity is None:
            capacity = max(1, text.numel() // 2 + 1)
        dev = text.device
        values = torch.empty(capacity, dtype=dtype, device=dev)
        status = torch.empty(capacity, dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        n = self.parse_into(text, values, status, count, stream=stream, sync=True)
        if n == FFP_E_CAPACITY:
            total = int(count.item())
            return self.parse(text, dtype, capacity=total, stream=stream)
        check(n, "parse")
        return values[:n], status[:n]


# ---------------------------------------------------------------------------
# batched calls: job tables and captured graphs
# ---------------------------------------------------------------------------

class JobTable:
    """ffp_job records for a list of (text, values, status) device tensors,
    kept both on the host (ctypes array) and on the device (uint8 tensor)."""

    def __init__(self, texts, values, statuses, device):
        import torch
        n = len(texts)
        self.n = n
        self.host = (ffp_job * n)()
        for i, (t, v, st) in enumerate(zip(texts, values, statuses)):
            self.host[i].text = t.data_ptr() if t.numel() else 0
            self.host[i].nbytes = t.numel()
            self.host[i].values = v.data_ptr()
            self.host[i].status = st.data_ptr()
            self.host[i].capacity = min(v.numel(), st.numel())
            self.host[i].dtype = {torch.float64: DTYPE_F64, torch.float32: DTYPE_F32,
                                  torch.float16: DTYPE_F16,
                                  torch.bfloat16: DTYPE_BF16}[v.dtype]
            self.host[i].err = 0
            self.host[i].count = 0
        raw = bytes(self.host)
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.total_bytes = sum(t.numel() for t in texts)

    def upload(self):
        import torch
        raw = bytes(self.host)
        self.dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))

    def download(self):
        raw = self.dev.cpu().numpy().tobytes()
        ctypes.memmove(ctypes.addressof(self.host), raw, len(raw))
        return [(self.host[i].count, self.host[i].err) for i in range(self.n)]


class BatchGraph:
    """A batched parse captured into a HIP graph (ffp_batch_graph_*)."""

    def __init__(self, ctx, table, max_total_bytes):
        out = _P()
        check(load().ffp_batch_graph_create(ctx.handle, table.dev.data_ptr(), table.n,
                                            max_total_bytes, ctypes.byref(out)),
              "ffp_batch_graph_create")
        self.handle = out
        _live["graph"].add(self)

    def launch(self, stream=None):
        check(load().ffp_batch_graph_launch(self.handle, _stream_handle(stream)),
              "ffp_batch_graph_launch")

    def close(self):
        if self.handle:
            load().ffp_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _finalize is not None:  # None once the module is torn down
            _finalize(self)


# ---------------------------------------------------------------------------
# serving (ffp_server_*)
# ---------------------------------------------------------------------------

def clock_ns() -> int:
    """CLOCK_MONOTONIC nanoseconds, the clock of the server's timestamps."""
    return load().ffp_clock_ns()


class Server:
    """A request server (continuous batching) created from a Context."""

    def __init__(self, ctx, hbm_budget_bytes=0, max_batch_bytes=0, max_inflight=0, streams=0,
                 max_batch_jobs=0, mode=FFP_SERVE_BATCHED, use_graph=False, spin_us=0):
        o = ffp_server_options()
        o.spin_us = spin_us
        o.hbm_budget_bytes = hbm_budget_bytes
        o.max_batch_bytes = max_batch_bytes
        o.max_inflight = max_inflight
        o.streams = streams
        o.max_batch_jobs = max_batch_jobs
        o.mode = mode
        o.use_graph = 1 if use_graph else 0
        out = _P()
        check(load().ffp_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(out)),
              "ffp_server_create")
        self.handle = out
        _live["server"].add(self)

    def submit_ptr(self, ptr, nbytes, on_device, dtype=DTYPE_F64, arrival_ns=0):
        """Submit raw memory; returns the ticket or raises FFPError."""
        t = ctypes.c_uint64()
        check(load().ffp_server_submit(self.handle, ptr, nbytes, 1 if on_device else 0, dtype,
                                       arrival_ns, ctypes.byref(t)), "ffp_server_submit")
        return t.value

    def submit(self, text, dtype=DTYPE_F64, arrival_ns=0):
        """Submit a contiguous uint8 tensor (device, or pinned host)."""
        return self.submit_ptr(text.data_ptr() if text.numel() else 0, text.numel(),
                               text.is_cuda, dtype, arrival_ns)

    def poll(self, ticket):
        r = ffp_result()
        rc = check(load().ffp_server_poll(self.handle, ticket, ctypes.byref(r)), "poll")
        return r if rc == 1 else None

    def wait(self, ticket):
        r = ffp_result()
        check(load().ffp_server_wait(self.handle, ticket, ctypes.byref(r)), "wait")
        return r

    def copy_result(self, ticket, values, status, stream=None):
        """ffp_server_copy_result into caller tensors (device or pinned host),
        stream-ordered on `stream`; the request may be released right after."""
        n = min(values.numel(), status.numel())
        check(load().ffp_server_copy_result(self.handle, ticket, values.data_ptr(),
                                            status.data_ptr(), n, _stream_handle(stream)),
              "copy_result")

    def result_tensors(self, ticket, device, stream=None):
        """Copies a done request's values and status into new device tensors."""
        import torch
        r = self.wait(ticket)
        dt = {DTYPE_F64: torch.float64, DTYPE_F32: torch.float32, DTYPE_F16: torch.float16,
              DTYPE_BF16: torch.bfloat16}[r.dtype]
        values = torch.empty(r.count, dtype=dt, device=device)
        status = torch.empty(r.count, dtype=torch.uint8, device=device)
        if r.count:
            check(load().ffp_server_copy_result(self.handle, ticket, values.data_ptr(),
                                                status.data_ptr(), r.count,
                                                _stream_handle(stream)), "copy_result")
        return r, values, status

    def release(self, ticket):
        check(load().ffp_server_release(self.handle, ticket), "release")

    def replay(self, ptrs, sizes, on_device, dtypes, arrival_ns, dst_values=None,
               dst_status=None, dst_capacity=None):
        """Replays an arrival trace (ffp_server_replay); returns a numpy
        structured array of per-request results.  With dst_* (per-request
        pointers and capacities) each request's results are copied there."""
        import numpy as np
        n = len(ptrs)
        req = np.zeros(n, dtype=np.dtype([("text", "<u8"), ("nbytes", "<u8"),
                                          ("on_device", "<i4"), ("dtype", "<i4"),
                                          ("arrival_ns", "<u8"), ("dst_values", "<u8"),
                                          ("dst_status", "<u8"), ("dst_capacity", "<u8")]))
        req["text"] = ptrs
        req["nbytes"] = sizes
        req["on_device"] = on_device
        req["dtype"] = dtypes
        req["arrival_ns"] = arrival_ns
        if dst_values is not None:
            req["dst_values"] = dst_values
            req["dst_status"] = dst_status
            req["dst_capacity"] = dst_capacity
        out = np.zeros(n, dtype=np.dtype([("t_arrive_ns", "<u8"), ("t_launch_ns", "<u8"),
                                          ("t_done_ns", "<u8"), ("count", "<u8"),
                                          ("err", "<i4"), ("batch_jobs", "<u4")]))
        assert req.itemsize == ctypes.sizeof(ffp_replay_request)
        assert out.itemsize == ctypes.sizeof(ffp_replay_result)
        check(load().ffp_server_replay(self.handle, req.ctypes.data, n, out.ctypes.data),
              "ffp_server_replay")
        return out

    def stats(self):
        st = ffp_server_stats()
        check(load().ffp_server_stats_read(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ffp_server_stats._fields_}

    def close(self):
        if self.handle:
            load().ffp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _finalize is not None:  # None once the module is torn down
            _finalize(self)
