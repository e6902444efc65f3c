"""libdedisp for MI355X: brute-force incoherent de-dispersion (Magro et al. 2011).

A thin ctypes binding over the C ABI in include/dedisp.h.  Every step of the
computation runs in the HIP library; this module only marshals arguments.
PyTorch supplies device memory (tensors) and streams.  If the library has
not been built, every call raises `LibraryMissing`: there is no CPU fallback.

    import torch, paper_1107_2516_amd as dd
    plan = dd.Plan(nchans=1024, f_top=1510.0, df=296/1024, t_samp=64e-6, dms=dms)
    out = plan.execute(x)        # x: [nchans, nsamp] float32/float16/uint8 on cuda
"""
import ctypes
import os
import re
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdedisp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "dedisp.h")

DD_OK = 0
DD_ERR_INVALID_ARG = -1
DD_ERR_DTYPE = -2
DD_ERR_NSAMP = -3
DD_ERR_OOM = -4
DD_ERR_HIP = -5
DD_ERR_AGAIN = -6
DD_ERR_TOO_LARGE = -7
DD_ERR_NOT_FOUND = -8
DD_ERR_NOT_IMPLEMENTED = -9
DD_ERR_STATE = -10

DD_U8, DD_F16, DD_F32, DD_I32 = 1, 2, 3, 4


class LibraryMissing(RuntimeError):
    pass


class DedispError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class TileConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("dms_per_wave", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("tsamp_per_lane", ctypes.c_int32),
                ("chans_per_stage", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_in", ctypes.c_void_p), ("nsamp", ctypes.c_int64),
                ("in_stride", ctypes.c_int64), ("d_out", ctypes.c_void_p),
                ("out_stride", ctypes.c_int64)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("in_t", ctypes.c_int), ("out_t", ctypes.c_int), ("max_inflight", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("nstreams", ctypes.c_int32),
                ("host_staging_bytes", ctypes.c_size_t)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("beam", ctypes.c_int32), ("status", ctypes.c_int32),
                ("seq", ctypes.c_int64), ("t_first", ctypes.c_int64), ("nout", ctypes.c_int64),
                ("d_out", ctypes.c_void_p), ("out_stride", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None
_lock = threading.Lock()
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

_SIGS = {
    "dd_plan_create": [_I32, _D, _D, _D, _P, _I32, _PP],
    "dd_plan_create_from_delays": [_I32, _I32, _P, _PP],
    "dd_plan_info": [_P, _P, _P, _P],
    "dd_delay_table": [_P, _P],
    "dd_plan_destroy": [_P],
    "dd_execute": [_P, _P, ctypes.c_int, _I64, _I64, _P, ctypes.c_int, _I64, _P],
    "dd_batch_create": [_P, _I32, ctypes.c_int, ctypes.c_int, _PP],
    "dd_batch_update": [_P, _P, _I32],
    "dd_batch_launch": [_P, _P],
    "dd_batch_destroy": [_P],
    "dd_batch_info": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(TileConfig)],
    "dd_batch_autotune": [_P, _P, ctypes.POINTER(TileConfig), ctypes.POINTER(ctypes.c_float)],
    "dd_batch_set_tile": [_P, ctypes.POINTER(TileConfig)],
    "dd_execute_tiled": [_P, _P, ctypes.c_int, _I64, _I64, _P, ctypes.c_int, _I64,
                         ctypes.POINTER(TileConfig), _P],
    "dd_autotune": [_P, ctypes.c_int, _I64, _P, ctypes.POINTER(TileConfig), ctypes.POINTER(ctypes.c_float)],
    "dd_tile_for": [_P, ctypes.c_int, _I64, ctypes.POINTER(TileConfig)],
    "dd_serve_create": [ctypes.POINTER(ServeConfig), _P, ctypes.c_size_t, _PP],
    "dd_serve_add_beam": [_P, _P, _I64, ctypes.POINTER(_I32)],
    "dd_serve_submit": [_P, _I32, _P, _I64, _I64, _I64, ctypes.POINTER(ctypes.c_uint64)],
    "dd_serve_poll": [_P, ctypes.POINTER(Result), _I32, ctypes.POINTER(_I32)],
    "dd_serve_release": [_P, ctypes.c_uint64],
    "dd_serve_drain": [_P],
    "dd_serve_destroy": [_P],
    "dd_serve_stats": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                       ctypes.POINTER(ctypes.c_size_t)],
    "dd_detect": [_P, ctypes.c_int, _I32, _I64, _I64, ctypes.c_float, _I32, _P, _P, _I64, _P, _P],
    "dd_detect_noalloc": [_P, ctypes.c_int, _I32, _I64, _I64, ctypes.c_float, _I32, _P, _I64, _P,
                          _P],
    "dd_corner_turn": [_P, ctypes.c_int, _I64, _I32, _I64, _I32, _P, _I64, _P],
    "dd_channelise": [_P, _I64, _I32, _I64, _I32, _P, _I64, _P],
    "dd_subband_plan_create": [_I32, _D, _D, _D, _I32, _P, _I32, _PP],
    "dd_subband_plan_info": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)],
    "dd_subband_dms": [_P, _P, _P],
    "dd_subband_sizes": [_P, _I64, _P, ctypes.POINTER(ctypes.c_size_t)],
    "dd_subband_execute": [_P, _P, _I64, _I64, _P, _I64, _P, ctypes.c_size_t, _P],
    "dd_subband_plan_destroy": [_P],
    "dd_jump_table_build": [_P, _I64, _I32, _I32, _I32, _P],
    "dd_jump_table_check": [_P, _P, _I64, _I32, _I32, _I32],
    "dd_pair_table_sizes": [_P, _I32, _I32, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "dd_pair_table_build": [_P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P],
    "dd_pair_table_check": [_P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P],
}


def lib():
    """The loaded libdedisp (raises LibraryMissing if it was never built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run `python -m paper_1107_2516_amd.build` "
                "(or __graft_entry__.build()). There is no CPU fallback.")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.dd_status_str.argtypes = [ctypes.c_int]
        L.dd_status_str.restype = ctypes.c_char_p
        L.dd_last_error.argtypes = []
        L.dd_last_error.restype = ctypes.c_char_p
        L.dd_version.argtypes = []
        L.dd_version.restype = ctypes.c_char_p
        _lib = L
        return L


def header_symbols():
    """Every function the C header declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z0-9_]+)\s*\(", txt)))


def status_str(status: int) -> str:
    return lib().dd_status_str(int(status)).decode()


def last_error() -> str:
    return lib().dd_last_error().decode()


def version() -> str:
    return lib().dd_version().decode()


def _check(status):
    if status != DD_OK:
        raise DedispError(status, last_error())


def _torch():
    import torch
    return torch


def dtype_code(dtype) -> int:
    torch = _torch()
    m = {torch.float32: DD_F32, torch.float16: DD_F16, torch.uint8: DD_U8, torch.int32: DD_I32}
    if dtype not in m:
        raise DedispError(DD_ERR_DTYPE, f"unsupported dtype {dtype}")
    return m[dtype]


def out_dtype_for(in_dtype):
    torch = _torch()
    return torch.int32 if in_dtype == torch.uint8 else torch.float32


def stream_handle(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Plan:
    """A de-dispersion plan: the FP64 delay table of section 3 ("Shifts")."""

    def __init__(self, nchans=None, f_top=None, df=None, t_samp=None, dms=None, *, _handle=None):
        L = lib()
        if _handle is not None:
            self._h = _handle
        else:
            dms = np.ascontiguousarray(np.asarray(dms, dtype=np.float64).reshape(-1))
            h = ctypes.c_void_p()
            _check(L.dd_plan_create(int(nchans), float(f_top), float(df), float(t_samp),
                                    dms.ctypes.data if dms.size else None, int(dms.size),
                                    ctypes.byref(h)))
            self._h = h
        n, d, m = _I32(), _I32(), _I32()
        _check(L.dd_plan_info(self._h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(m)))
        self.nchans, self.ndms, self.max_shift = n.value, d.value, m.value

    @classmethod
    def from_delays(cls, delays):
        t = np.ascontiguousarray(np.asarray(delays), dtype=np.int32)
        if t.ndim != 2:
            raise DedispError(DD_ERR_INVALID_ARG, "delays must be [ndms, nchans]")
        h = ctypes.c_void_p()
        _check(lib().dd_plan_create_from_delays(int(t.shape[1]), int(t.shape[0]), t.ctypes.data,
                                                ctypes.byref(h)))
        return cls(_handle=h)

    @property
    def handle(self):
        return self._h

    def delay_table(self) -> np.ndarray:
        out = np.empty((self.ndms, self.nchans), dtype=np.int32)
        _check(lib().dd_delay_table(self._h, out.ctypes.data))
        return out

    def nout(self, nsamp: int) -> int:
        return int(nsamp) - self.max_shift

    def execute(self, inp, out=None, stream=None):
        """De-disperse `inp` ([nchans, nsamp] on the GPU, rows may be padded)
        into `out` ([ndms, >= nout]); allocates `out` if not given."""
        torch = _torch()
        if inp.dim() != 2 or inp.shape[0] != self.nchans:
            raise DedispError(DD_ERR_INVALID_ARG, f"input must be [{self.nchans}, nsamp]")
        if inp.stride(1) != 1:
            raise DedispError(DD_ERR_INVALID_ARG, "time axis must be contiguous")
        nsamp = inp.shape[1]
        if out is None:
            out = torch.empty((self.ndms, max(self.nout(nsamp), 0)), dtype=out_dtype_for(inp.dtype),
                              device=inp.device)
        if out.dim() != 2 or out.stride(1) != 1 or out.shape[0] != self.ndms:
            raise DedispError(DD_ERR_INVALID_ARG, f"output must be [{self.ndms}, nout] row-major")
        if not inp.is_cuda or not out.is_cuda:
            raise DedispError(DD_ERR_INVALID_ARG, "tensors must be on the GPU")
        _check(lib().dd_execute(self._h, inp.data_ptr(), dtype_code(inp.dtype), nsamp,
                                inp.stride(0), out.data_ptr(), dtype_code(out.dtype),
                                out.stride(0), stream_handle(stream)))
        return out

    def execute_tiled(self, inp, tile, out=None, stream=None):
        """execute() with an explicit tile shape (a dict of TileConfig fields)."""
        torch = _torch()
        nsamp = inp.shape[1]
        if out is None:
            out = torch.empty((self.ndms, max(self.nout(nsamp), 0)), dtype=out_dtype_for(inp.dtype),
                              device=inp.device)
        cfg = TileConfig(**tile)
        _check(lib().dd_execute_tiled(self._h, inp.data_ptr(), dtype_code(inp.dtype), nsamp,
                                      inp.stride(0), out.data_ptr(), dtype_code(out.dtype),
                                      out.stride(0), ctypes.byref(cfg), stream_handle(stream)))
        return out

    def tile_for(self, in_dtype, nsamp):
        cfg = TileConfig()
        _check(lib().dd_tile_for(self._h, dtype_code(in_dtype), int(nsamp), ctypes.byref(cfg)))
        return cfg.as_dict()

    def autotune(self, in_dtype, nsamp, stream=None):
        cfg = TileConfig()
        ms = ctypes.c_float()
        _check(lib().dd_autotune(self._h, dtype_code(in_dtype), int(nsamp), stream_handle(stream),
                                 ctypes.byref(cfg), ctypes.byref(ms)))
        return cfg.as_dict(), ms.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_plan_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many beams de-dispersed by one persistent, graph-captured launch.

    beams: list of (plan, input tensor [nchans, nsamp], output tensor or None).
    All inputs share one dtype.  Outputs are allocated when None.
    """

    def __init__(self, beams):
        torch = _torch()
        if not beams:
            raise DedispError(DD_ERR_INVALID_ARG, "need at least one beam")
        self.plans = [b[0] for b in beams]
        self.inputs = [b[1] for b in beams]
        self.outputs = []
        for plan, x, o in beams:
            if o is None:
                o = torch.empty((plan.ndms, plan.nout(x.shape[1])), dtype=out_dtype_for(x.dtype),
                                device=x.device)
            self.outputs.append(o)
        self.in_dtype = self.inputs[0].dtype
        items = self._items()
        h = ctypes.c_void_p()
        _check(lib().dd_batch_create(items, len(items), dtype_code(self.in_dtype),
                                     dtype_code(out_dtype_for(self.in_dtype)), ctypes.byref(h)))
        self._h = h

    def _items(self):
        arr = (BatchItem * len(self.plans))()
        for i, (p, x, o) in enumerate(zip(self.plans, self.inputs, self.outputs)):
            if x.dtype != self.in_dtype:
                raise DedispError(DD_ERR_DTYPE, "all beams of a batch share one input dtype")
            if x.dim() != 2 or x.stride(1) != 1 or x.shape[0] != p.nchans:
                raise DedispError(DD_ERR_INVALID_ARG, "beam input must be [nchans, nsamp]")
            if o.dim() != 2 or o.stride(1) != 1 or o.shape[0] != p.ndms:
                raise DedispError(DD_ERR_INVALID_ARG, "beam output must be [ndms, nout]")
            arr[i] = BatchItem(p.handle.value if isinstance(p.handle, ctypes.c_void_p) else p.handle,
                               x.data_ptr(), x.shape[1], x.stride(0), o.data_ptr(), o.stride(0))
        return arr

    def update(self, inputs=None, outputs=None):
        """Point the batch at new tensors of the same shapes and strides."""
        if inputs is not None:
            self.inputs = list(inputs)
        if outputs is not None:
            self.outputs = list(outputs)
        items = self._items()
        _check(lib().dd_batch_update(self._h, items, len(items)))

    def launch(self, stream=None):
        _check(lib().dd_batch_launch(self._h, stream_handle(stream)))
        return self.outputs

    def info(self):
        n, g, cfg = _I32(), _I32(), TileConfig()
        _check(lib().dd_batch_info(self._h, ctypes.byref(n), ctypes.byref(g), ctypes.byref(cfg)))
        return {"work_items": n.value, "grid": g.value, "tile": cfg.as_dict()}

    def set_tile(self, tile):
        """Force one tile shape (a dict like info()["tile"]) for every beam."""
        cfg = TileConfig(int(tile["variant"]), int(tile["dms_per_wave"]), int(tile["waves"]),
                         int(tile["tsamp_per_lane"]), int(tile["chans_per_stage"]))
        _check(lib().dd_batch_set_tile(self._h, ctypes.byref(cfg)))

    def autotune(self, stream=None):
        cfg, ms = TileConfig(), ctypes.c_float()
        _check(lib().dd_batch_autotune(self._h, stream_handle(stream), ctypes.byref(cfg),
                                       ctypes.byref(ms)))
        return cfg.as_dict(), ms.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Streaming server: chunks of many beams, continuous batching on the GPU.

    arena: a uint8 CUDA tensor whose memory the server sub-allocates (beam
    rings, chunk staging and outputs); it must outlive the server.
    """

    def __init__(self, arena, in_dtype, max_inflight=8, queue_capacity=256, nstreams=4,
                 host_staging_bytes=0):
        self.arena = arena
        self.in_dtype = in_dtype
        self.out_dtype = out_dtype_for(in_dtype)
        cfg = ServeConfig(dtype_code(in_dtype), dtype_code(self.out_dtype), max_inflight,
                          queue_capacity, nstreams, host_staging_bytes)
        h = ctypes.c_void_p()
        _check(lib().dd_serve_create(ctypes.byref(cfg), arena.data_ptr(),
                                     arena.numel() * arena.element_size(), ctypes.byref(h)))
        self._h = h
        self.beams = []

    def add_beam(self, plan, max_chunk):
        b = _I32()
        _check(lib().dd_serve_add_beam(self._h, plan.handle, int(max_chunk), ctypes.byref(b)))
        self.beams.append(plan)
        return b.value

    def submit(self, beam, chunk: np.ndarray, seq):
        """Queue a host chunk [nchans, nsamp] (numpy array whose rows are
        contiguous; rows may be a stride apart, e.g. a column slice).
        Returns the ticket, or None when the server is full (DD_ERR_AGAIN)."""
        c = chunk
        if c.ndim != 2 or c.strides[1] != c.itemsize or c.strides[0] % c.itemsize:
            c = np.ascontiguousarray(c)
        t = ctypes.c_uint64()
        st = lib().dd_serve_submit(self._h, int(beam), c.ctypes.data, int(c.shape[1]),
                                   int(c.strides[0] // c.itemsize), int(seq), ctypes.byref(t))
        if st == DD_ERR_AGAIN:
            return None
        _check(st)
        return t.value

    def poll(self, max_results=64):
        arr = (Result * max_results)()
        n = _I32()
        _check(lib().dd_serve_poll(self._h, arr, max_results, ctypes.byref(n)))
        return [arr[i] for i in range(n.value)]

    def output(self, result):
        """The device output of a finished chunk as a tensor view into the
        arena, [ndms, nout] (valid until release)."""
        plan = self.beams[result.beam]
        if result.nout == 0:
            return None
        torch = _torch()
        esize = 4
        off = result.d_out - self.arena.data_ptr()
        n = (plan.ndms - 1) * result.out_stride + result.nout  # elements the rows span
        flat = self.arena[off: off + n * esize].view(self.out_dtype)
        return flat.as_strided((plan.ndms, result.nout), (result.out_stride, 1))

    def release(self, ticket):
        _check(lib().dd_serve_release(self._h, int(ticket)))

    def stats(self):
        p, i, f, z = _I32(), _I32(), _I32(), ctypes.c_size_t()
        _check(lib().dd_serve_stats(self._h, ctypes.byref(p), ctypes.byref(i), ctypes.byref(f),
                                    ctypes.byref(z)))
        return {"pending": p.value, "inflight": i.value, "finished": f.value,
                "largest_free": z.value}

    def drain(self):
        _check(lib().dd_serve_drain(self._h))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_serve_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# dd_event as a numpy record (24 bytes, the C layout)
EVENT_DTYPE = np.dtype([("dm_row", np.int32), ("width", np.int32), ("t", np.int64),
                        ("snr", np.float32), ("reserved", np.int32)])


def detect(out, nsigma, max_log2_width=6, max_events=1 << 20, stream=None):
    """Detection stage on a de-dispersed tensor out [ndms, nout] (float32 or
    int32, rows contiguous): per-row mean/sigma, boxcars of widths 1..2^k,
    events where a sample's best S/N >= nsigma.  Returns (events sorted by
    (dm_row, t) as a numpy record array, per-row stats tensor [ndms, 2]
    (mu, sigma), total number of events found)."""
    torch = _torch()
    if out.dim() != 2 or out.stride(1) != 1:
        raise DedispError(DD_ERR_INVALID_ARG, "out must be [ndms, nout] with contiguous rows")
    ndms, nout = out.shape
    stats = torch.empty((ndms, 2), dtype=torch.float64, device=out.device)
    ev = torch.empty((max(1, max_events), EVENT_DTYPE.itemsize), dtype=torch.uint8,
                     device=out.device)
    count = torch.zeros(1, dtype=torch.int64, device=out.device)
    _check(lib().dd_detect(out.data_ptr(), dtype_code(out.dtype), ndms, nout, out.stride(0),
                           float(nsigma), int(max_log2_width), stats.data_ptr(), ev.data_ptr(),
                           int(max_events), count.data_ptr(), stream_handle(stream)))
    s = torch.cuda.current_stream() if stream is None else stream
    s.synchronize()
    n = int(count.item())
    k = min(n, max_events)
    host = ev[:k].cpu().numpy().reshape(-1).view(EVENT_DTYPE)
    host = host[np.lexsort((host["t"], host["dm_row"]))]
    return host, stats, n


def detect_noalloc(out, nsigma, events, count, max_log2_width=6, stream=None):
    """dd_detect_noalloc: detection into caller tensors `events` (uint8
    [max_events, 24]) and `count` (int64 [1]) on the device, with the per-row
    statistics in the library's static device array; queues the work on
    `stream` and returns without waiting or allocating."""
    if out.dim() != 2 or out.stride(1) != 1:
        raise DedispError(DD_ERR_INVALID_ARG, "out must be [ndms, nout] with contiguous rows")
    if events.dim() != 2 or events.shape[1] != EVENT_DTYPE.itemsize or not events.is_contiguous():
        raise DedispError(DD_ERR_INVALID_ARG, "events must be contiguous [max_events, 24] bytes")
    ndms, nout = out.shape
    _check(lib().dd_detect_noalloc(out.data_ptr(), dtype_code(out.dtype), ndms, nout,
                                   out.stride(0), float(nsigma), int(max_log2_width),
                                   events.data_ptr(), int(events.shape[0]), count.data_ptr(),
                                   stream_handle(stream)))


def events_from_device(events, count):
    """Host copy of the first min(count, capacity) events, sorted by (dm_row, t),
    and the total count."""
    n = int(count.item())
    k = min(n, events.shape[0])
    host = events[:k].cpu().numpy().reshape(-1).view(EVENT_DTYPE)
    return host[np.lexsort((host["t"], host["dm_row"]))], n


def corner_turn(spectra, flip=False, out=None, stream=None):
    """Time-ordered spectra [nsamp, nchans] (uint8, float16 or float32 CUDA
    tensor with contiguous rows) -> channel-ordered rows [nchans, nsamp]
    (channels reversed when flip)."""
    torch = _torch()
    if spectra.dim() != 2 or spectra.stride(1) != 1:
        raise DedispError(DD_ERR_INVALID_ARG, "spectra must be [nsamp, nchans] with contiguous rows")
    nsamp, nchans = spectra.shape
    if out is None:
        out = torch.empty((nchans, nsamp), dtype=spectra.dtype, device=spectra.device)
    if out.dim() != 2 or out.stride(1) != 1 or tuple(out.shape) != (nchans, nsamp):
        raise DedispError(DD_ERR_INVALID_ARG, "out must be [nchans, nsamp] with contiguous rows")
    _check(lib().dd_corner_turn(spectra.data_ptr(), dtype_code(spectra.dtype), nsamp, nchans,
                                spectra.stride(0), 1 if flip else 0, out.data_ptr(), out.stride(0),
                                stream_handle(stream)))
    return out


class SubbandPass(ctypes.Structure):
    _fields_ = [("dm_lo", ctypes.c_double), ("dm_hi", ctypes.c_double), ("ddm", ctypes.c_double),
                ("dsub", ctypes.c_double), ("bin", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SubbandPlan:
    """Section 3.2 subband de-dispersion over a survey plan of passes
    (dm_lo, dm_hi, ddm, dsub, bin), FP32 in and out."""

    def __init__(self, nchans, f_top, df, t_samp, nsub, passes):
        arr = (SubbandPass * len(passes))()
        for i, (lo, hi, ddm, dsub, b) in enumerate(passes):
            arr[i] = SubbandPass(float(lo), float(hi), float(ddm), float(dsub), int(b), 0)
        h = ctypes.c_void_p()
        _check(lib().dd_subband_plan_create(int(nchans), float(f_top), float(df), float(t_samp),
                                            int(nsub), arr, len(passes), ctypes.byref(h)))
        self._h = h
        n, npass = _I32(), _I32()
        _check(lib().dd_subband_plan_info(h, ctypes.byref(n), ctypes.byref(npass)))
        self.ndms, self.npass = n.value, npass.value
        self.nchans = int(nchans)

    def dms(self):
        d = np.zeros(self.ndms, dtype=np.float64)
        p = np.zeros(self.ndms, dtype=np.int32)
        _check(lib().dd_subband_dms(self._h, d.ctypes.data, p.ctypes.data))
        return d, p

    def sizes(self, nsamp):
        n = np.zeros(self.npass, dtype=np.int64)
        ws = ctypes.c_size_t()
        _check(lib().dd_subband_sizes(self._h, int(nsamp), n.ctypes.data, ctypes.byref(ws)))
        return n, ws.value

    def execute(self, x, out=None, workspace=None, stream=None):
        """x [nchans, nsamp] float32 CUDA tensor (contiguous rows).  Returns
        (out [ndms, max nout], nout per pass); row r is valid up to the nout
        of its pass."""
        torch = _torch()
        if x.dim() != 2 or x.stride(1) != 1 or x.shape[0] != self.nchans or x.dtype != torch.float32:
            raise DedispError(DD_ERR_INVALID_ARG, "x must be float32 [nchans, nsamp]")
        nsamp = x.shape[1]
        nout, ws = self.sizes(nsamp)
        if out is None:
            out = torch.zeros((self.ndms, int(nout.max())), dtype=torch.float32, device=x.device)
        if workspace is None:
            workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=x.device)
        _check(lib().dd_subband_execute(self._h, x.data_ptr(), nsamp, x.stride(0), out.data_ptr(),
                                        out.stride(0), workspace.data_ptr(),
                                        workspace.numel(), stream_handle(stream)))
        return out, nout

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_subband_plan_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def channelise(volt, nfft, out=None, stream=None):
    """Section 5 front end: volt [nsamp, nsub] complex64 CUDA tensor (one
    spectrum of coarse subbands per time sample) -> channel-ordered power
    [nsub*nfft, nsamp // nfft] float32 (FFT of nfft samples per subband)."""
    torch = _torch()
    if volt.dim() != 2 or volt.dtype != torch.complex64 or volt.stride(1) != 1:
        raise DedispError(DD_ERR_INVALID_ARG, "volt must be complex64 [nsamp, nsub], contiguous rows")
    nsamp, nsub = volt.shape
    nt = nsamp // int(nfft)
    if out is None:
        out = torch.empty((nsub * int(nfft), nt), dtype=torch.float32, device=volt.device)
    if out.dim() != 2 or out.stride(1) != 1 or tuple(out.shape) != (nsub * int(nfft), nt):
        raise DedispError(DD_ERR_INVALID_ARG, "out must be [nsub*nfft, nsamp//nfft]")
    _check(lib().dd_channelise(volt.data_ptr(), nsamp, nsub, volt.stride(0), int(nfft),
                               out.data_ptr(), out.stride(0), stream_handle(stream)))
    return out
