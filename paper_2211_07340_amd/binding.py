"""ctypes binding of libsdtw.so: same names as the C ABI, argument marshalling only.

Tensors are torch tensors; device pointers are ``tensor.data_ptr()`` and the
stream is ``torch.cuda.current_stream().cuda_stream`` unless one is given.
If the library is missing every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

F32, I16 = 0, 1
_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EBUDGET", 4: "EDEVICE", 5: "ESTATE"}
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsdtw.so")
_lib = None


class SdtwError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.code = _STATUS.get(status, str(status))
        super().__init__(f"{self.code}: {message}")


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libsdtw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = C.CDLL(_LIB_PATH)
    p, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "sdtw_last_error": ([], C.c_char_p),
        "sdtw_version": ([], C.c_int),
        "sdtw_prepare_reference": ([p, i64, p, C.c_int, dbl, p, p, p, p], C.c_int),
        "sdtw_prepare_queries": ([p, p, i32, dbl, p, p, p, p], C.c_int),
        "sdtw_load_reference": ([p, i64, C.c_int, C.c_int, p, C.POINTER(p)], C.c_int),
        "sdtw_reference_info": ([p, C.POINTER(i64), C.POINTER(C.c_int)], C.c_int),
        "sdtw_free_reference": ([p], C.c_int),
        "sdtw_plan_create": ([p, i32, C.c_int, C.POINTER(p)], C.c_int),
        "sdtw_plan_info": ([p, C.POINTER(i32), C.POINTER(C.c_int), C.POINTER(i32)], C.c_int),
        "sdtw_plan_set_config": ([p, C.c_int, C.c_int, C.c_int, C.c_int, i32], C.c_int),
        "sdtw_plan_get_config": ([p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(i32)], C.c_int),
        "sdtw_plan_destroy": ([p], C.c_int),
        "sdtw_plan_autotune": ([p, p, p, p, p, i64, p], C.c_int),
        "sdtw_plan_use_tuned": ([p, p, C.POINTER(C.c_int)], C.c_int),
        "sdtw_align_batch": ([p, p, p, p, p, p], C.c_int),
        "sdtw_align_one": ([p, p, i32, p, p, p], C.c_int),
        "sdtw_align_one_wide": ([p, p, i32, C.c_int, p, p, p], C.c_int),
        "sdtw_align_one_wide_noalloc": ([p, p, i32, C.c_int, p, p, p], C.c_int),
        "sdtw_detect_events": ([p, p, i32, i32, i32, p, p, p], C.c_int),
        "sdtw_detect_events_prefix": ([p, p, p, i32, i32, i32, p, p, p], C.c_int),
        "sdtw_event_state_bytes": ([], C.c_int64),
        "sdtw_event_state_init": ([p, p, i32, p], C.c_int),
        "sdtw_detect_events_continue": ([p, p, p, p, i32, i32, i32, p, p, p], C.c_int),
        "sdtw_prepare_queries_ex": ([p, p, i32, dbl, p, p, p, p, p, p], C.c_int),
        "sdtw_stream_set_config": ([p, C.c_int, C.c_int], C.c_int),
        "sdtw_row_pool_trim": ([], C.c_int),
        "sdtw_stream_best_two": ([p, i32, i32, p, p, p, p, p], C.c_int),
        "sdtw_set_row_budget": ([i64], C.c_int),
        "sdtw_row_budget_info": ([C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)], C.c_int),
        "sdtw_stream_open": ([p, C.POINTER(p)], C.c_int),
        "sdtw_stream_info": ([p, C.POINTER(i32), C.POINTER(i64)], C.c_int),
        "sdtw_stream_close": ([p], C.c_int),
        "sdtw_stream_copy_row": ([p, p, p], C.c_int),
        "sdtw_stream_extend": ([p, i32, p, p, p, p, p], C.c_int),
        "sdtw_stream_extend_wide": ([p, p, i32, C.c_int, p, p, p], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().sdtw_last_error().decode(errors="replace")
        raise SdtwError(status, msg)


def version() -> int:
    return load_library().sdtw_version()


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev(t, dtype=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _offsets_host(offsets) -> np.ndarray:
    if hasattr(offsets, "detach"):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(offsets, dtype=np.int64)


# ---------------------------------------------------------------------------
# preparation
# ---------------------------------------------------------------------------

def prepare_reference(genome, table, k: int = 6, scale: float = 64.0, stream=None):
    """Section 4.1 reference preparation on the device.

    genome: uint8 device tensor (A=0 C=1 G=2 T=3); table: float32 [4**k].
    Returns (z float32[2(L-k+1)], codes int16[...], nsat int64[1]) device tensors.
    """
    torch = _torch()
    lib = load_library()
    L = genome.numel()
    n = 2 * (L - k + 1)
    if n < 2:
        raise ValueError("genome shorter than k")
    z = torch.empty(n, dtype=torch.float32, device=genome.device)
    codes = torch.empty(n, dtype=torch.int16, device=genome.device)
    nsat = torch.empty(1, dtype=torch.int64, device=genome.device)
    _check(lib.sdtw_prepare_reference(_dev(genome, torch.uint8, "genome"), L,
                                      _dev(table, torch.float32, "table"), int(k), float(scale),
                                      _dev(z), _dev(codes), _dev(nsat), _stream(stream)))
    return z, codes, nsat


def prepare_queries(raw, offsets, scale: float = 64.0, stream=None):
    """Section 4.1 per-read normalisation and scaling on the device.

    raw: float32 device tensor (CSR values); offsets: int64 device tensor [nq+1].
    Returns (z float32, codes int16, nsat int64[1]) device tensors.
    """
    torch = _torch()
    lib = load_library()
    nq = offsets.numel() - 1
    z = torch.empty_like(raw)
    codes = torch.empty(raw.numel(), dtype=torch.int16, device=raw.device)
    nsat = torch.empty(1, dtype=torch.int64, device=raw.device)
    _check(lib.sdtw_prepare_queries(_dev(raw, torch.float32, "raw"),
                                    _dev(offsets, torch.int64, "offsets"), nq, float(scale),
                                    _dev(z), _dev(codes), _dev(nsat), _stream(stream)))
    return z, codes, nsat


def prepare_queries_ex(raw, offsets, scale: float = 64.0, stats_in=None, stream=None):
    """sdtw_prepare_queries_ex: as prepare_queries, with fixed per-read
    statistics (float64 device tensor [nq, 2] of (mean, sd)) if given.
    Returns (z, codes, nsat, stats) where stats are the (mean, sd) applied."""
    torch = _torch()
    lib = load_library()
    nq = offsets.numel() - 1
    z = torch.empty_like(raw)
    codes = torch.empty(raw.numel(), dtype=torch.int16, device=raw.device)
    nsat = torch.empty(1, dtype=torch.int64, device=raw.device)
    stats = torch.empty((nq, 2), dtype=torch.float64, device=raw.device)
    sin = None if stats_in is None else _dev(stats_in, torch.float64, "stats_in")
    _check(lib.sdtw_prepare_queries_ex(_dev(raw, torch.float32, "raw"),
                                       _dev(offsets, torch.int64, "offsets"), nq, float(scale),
                                       sin, _dev(stats), _dev(z), _dev(codes), _dev(nsat),
                                       _stream(stream)))
    return z, codes, nsat, stats


# ---------------------------------------------------------------------------
# reference and plans
# ---------------------------------------------------------------------------

class Reference:
    """Device copy of a prepared reference signal (sdtw_load_reference)."""

    def __init__(self, values, stream=None):
        torch = _torch()
        lib = load_library()
        if values.dtype == torch.int16:
            self.dtype = I16
        elif values.dtype == torch.float32:
            self.dtype = F32
        else:
            raise ValueError("reference must be int16 or float32")
        values = values.contiguous()
        self.n = values.numel()
        h = C.c_void_p()
        _check(lib.sdtw_load_reference(C.c_void_p(values.data_ptr()), self.n, self.dtype,
                                       1 if values.is_cuda else 0, _stream(stream),
                                       C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise SdtwError(5, "reference is closed")
        return self._h

    def close(self):
        if self._h is not None:
            _check(load_library().sdtw_free_reference(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Validated, longest-first batch layout (sdtw_plan_create)."""

    def __init__(self, offsets, dtype: int):
        lib = load_library()
        offs = _offsets_host(offsets)
        self.offsets = offs
        self.nq = offs.size - 1
        self.dtype = dtype
        h = C.c_void_p()
        _check(lib.sdtw_plan_create(offs.ctypes.data_as(C.c_void_p), self.nq, dtype,
                                    C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise SdtwError(5, "plan is closed")
        return self._h

    def set_config(self, strip: int = 0, chains: int = 0, waves_per_cu: int = 0,
                   bands: int = 0, band_rows: int = -1):
        """sdtw_plan_set_config; 0 (band_rows: -1) keeps a setting."""
        _check(load_library().sdtw_plan_set_config(self.handle, strip, chains, bands,
                                                   waves_per_cu, band_rows))

    @property
    def config(self):
        """dict(strip, chains, bands, waves_per_cu, band_rows)"""
        s, k, b, w, r = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int32()
        _check(load_library().sdtw_plan_get_config(self.handle, C.byref(s), C.byref(k),
                                                   C.byref(b), C.byref(w), C.byref(r)))
        return {"strip": s.value, "chains": k.value, "bands": b.value,
                "waves_per_cu": w.value, "band_rows": r.value}

    def close(self):
        if self._h is not None:
            _check(load_library().sdtw_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _outputs(nq, dtype, device, cost, end):
    torch = _torch()
    if cost is None:
        cost = torch.empty(nq, dtype=torch.int32 if dtype == I16 else torch.float32,
                           device=device)
    if end is None:
        end = torch.empty(nq, dtype=torch.int32, device=device)
    return cost, end


def align_batch(ref: Reference, plan: Plan, q, cost=None, end=None, stream=None):
    """sdtw_align_batch: returns (cost, end) device tensors (int32/float32, int32)."""
    torch = _torch()
    qdt = torch.int16 if plan.dtype == I16 else torch.float32
    cost, end = _outputs(plan.nq, plan.dtype, q.device, cost, end)
    _check(load_library().sdtw_align_batch(ref.handle, plan.handle, _dev(q, qdt, "q"),
                                           _dev(cost), _dev(end, torch.int32, "end"),
                                           _stream(stream)))
    return cost, end


def autotune(ref: Reference, plan: Plan, q, max_columns: int = 1 << 17, stream=None):
    """sdtw_plan_autotune: time the candidate configurations on this batch
    (first max_columns reference columns), keep the fastest on the plan;
    returns plan.config.  Synchronises the stream."""
    torch = _torch()
    qdt = torch.int16 if plan.dtype == I16 else torch.float32
    cost, end = _outputs(plan.nq, plan.dtype, q.device, None, None)
    _check(load_library().sdtw_plan_autotune(ref.handle, plan.handle, _dev(q, qdt, "q"),
                                             _dev(cost), _dev(end, torch.int32, "end"),
                                             int(max_columns), _stream(stream)))
    return plan.config


def use_tuned(ref: Reference, plan: Plan) -> bool:
    """sdtw_plan_use_tuned: apply an earlier autotune result for this shape."""
    found = C.c_int()
    _check(load_library().sdtw_plan_use_tuned(ref.handle, plan.handle, C.byref(found)))
    return bool(found.value)


def align_one(ref: Reference, q, cost=None, end=None, stream=None):
    """sdtw_align_one (single-wave kernel, one read per launch)."""
    torch = _torch()
    qdt = torch.int16 if ref.dtype == I16 else torch.float32
    cost, end = _outputs(1, ref.dtype, q.device, cost, end)
    _check(load_library().sdtw_align_one(ref.handle, _dev(q, qdt, "q"), q.numel(), _dev(cost),
                                         _dev(end, torch.int32, "end"), _stream(stream)))
    return cost, end


def detect_events(raw, offsets, trim: int = 50, keep: int = 250, events=None, counts=None,
                  stream=None):
    """sdtw_detect_events: (events float32 [nreads, keep], counts int32
    [nreads]) device tensors from raw samples (device float32) and int64
    device offsets; ``events`` / ``counts`` may be given (preallocated)."""
    torch = _torch()
    nreads = offsets.numel() - 1
    if nreads < 1:
        raise ValueError("no reads")
    ev = events if events is not None else torch.empty((nreads, keep), dtype=torch.float32,
                                                       device=raw.device)
    cnt = counts if counts is not None else torch.empty(nreads, dtype=torch.int32,
                                                        device=raw.device)
    if ev.numel() != nreads * keep or cnt.numel() != nreads:
        raise ValueError("events must hold nreads * keep values and counts nreads")
    _check(load_library().sdtw_detect_events(_dev(raw, torch.float32, "raw"),
                                             _dev(offsets, torch.int64, "offsets"), nreads,
                                             int(trim), int(keep), _dev(ev), _dev(cnt),
                                             _stream(stream)))
    return ev, cnt


def detect_events_prefix(raw, ranges, firsts, max_first: int, keep: int, events=None,
                         counts=None, stream=None):
    """sdtw_detect_events_prefix: final events of reads still being received.
    ``ranges`` int64 [nreads, 2] (start, end) and ``firsts`` int32 [nreads]
    device tensors; returns (events float32 [nreads, keep], counts int32)."""
    torch = _torch()
    nreads = firsts.numel()
    if nreads < 1 or ranges.numel() != 2 * nreads:
        raise ValueError("ranges must hold a (start, end) pair per read")
    ev = events if events is not None else torch.empty((nreads, keep), dtype=torch.float32,
                                                       device=raw.device)
    cnt = counts if counts is not None else torch.empty(nreads, dtype=torch.int32,
                                                        device=raw.device)
    _check(load_library().sdtw_detect_events_prefix(
        _dev(raw, torch.float32, "raw"), _dev(ranges, torch.int64, "ranges"),
        _dev(firsts, torch.int32, "firsts"), nreads, int(max_first), int(keep), _dev(ev),
        _dev(cnt), _stream(stream)))
    return ev, cnt


class EventStates:
    """Device memory for the detector state of `n` reads received chunk by
    chunk (sdtw_detect_events_continue)."""

    def __init__(self, n: int, device=None):
        torch = _torch()
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = int(load_library().sdtw_event_state_bytes())
        self.n = int(n)
        self.buf = torch.zeros(self.n * nbytes, dtype=torch.uint8, device=dev)

    def reset(self, slots, stream=None):
        """Start new reads on these slots (int32 device tensor)."""
        torch = _torch()
        if slots.numel() == 0:
            return
        _check(load_library().sdtw_event_state_init(_dev(self.buf), _dev(slots, torch.int32,
                                                                        "slots"),
                                                    slots.numel(), _stream(stream)))

    def detect(self, raw, ranges, slots, trim: int, keep: int, events=None, counts=None,
               stream=None):
        """(events float32 [n, keep], counts int32 [n]) for reads whose
        samples so far are ranges (int64 [n, 2]) on state slots (int32 [n])."""
        torch = _torch()
        n = slots.numel()
        if n < 1 or ranges.numel() != 2 * n:
            raise ValueError("ranges must hold a (start, end) pair per read")
        ev = events if events is not None else torch.empty((n, keep), dtype=torch.float32,
                                                           device=raw.device)
        cnt = counts if counts is not None else torch.empty(n, dtype=torch.int32,
                                                            device=raw.device)
        _check(load_library().sdtw_detect_events_continue(
            _dev(raw, torch.float32, "raw"), _dev(ranges, torch.int64, "ranges"),
            _dev(slots, torch.int32, "slots"), _dev(self.buf), n, int(trim), int(keep),
            _dev(ev), _dev(cnt), _stream(stream)))
        return ev, cnt


def align_one_wide(ref: Reference, q, cols: int = 0, cost=None, end=None, stream=None):
    """sdtw_align_one_wide (one int16 read over every compute unit)."""
    torch = _torch()
    cost, end = _outputs(1, ref.dtype, q.device, cost, end)
    _check(load_library().sdtw_align_one_wide(ref.handle, _dev(q, torch.int16, "q"), q.numel(),
                                              int(cols), _dev(cost),
                                              _dev(end, torch.int32, "end"), _stream(stream)))
    return cost, end


def align_one_wide_noalloc(ref: Reference, q, cost, end, cols: int = 0, stream=None):
    """sdtw_align_one_wide_noalloc: the same on the library's fixed scratch;
    the caller passes the outputs (int32[1] each), nothing is allocated."""
    torch = _torch()
    _check(load_library().sdtw_align_one_wide_noalloc(
        ref.handle, _dev(q, torch.int16, "q"), q.numel(), int(cols),
        _dev(cost, torch.int32, "cost"), _dev(end, torch.int32, "end"), _stream(stream)))
    return cost, end


# ---------------------------------------------------------------------------
# streaming extension
# ---------------------------------------------------------------------------

def set_row_budget(nbytes: int):
    """Byte budget of resident rows on the current device."""
    _check(load_library().sdtw_set_row_budget(int(nbytes)))


def stream_best_two(streams, window: int, stream=None):
    """sdtw_stream_best_two: (best_cost, best_end, second_cost, second_end)
    device tensors for the streams' resident rows."""
    torch = _torch()
    ns = len(streams)
    if ns == 0:
        raise ValueError("no streams")
    dt = streams[0].ref.dtype
    dev = torch.device("cuda", torch.cuda.current_device())
    cdt = torch.int32 if dt == I16 else torch.float32
    bc, sc = torch.empty(ns, dtype=cdt, device=dev), torch.empty(ns, dtype=cdt, device=dev)
    be, se = (torch.empty(ns, dtype=torch.int32, device=dev),
              torch.empty(ns, dtype=torch.int32, device=dev))
    arr = (C.c_void_p * ns)(*[s.handle for s in streams])
    _check(load_library().sdtw_stream_best_two(arr, ns, int(window), _dev(bc), _dev(be),
                                               _dev(sc), _dev(se), _stream(stream)))
    return bc, be, sc, se


def set_stream_config(strip: int = 0, bands: int = 0, ref: Reference | None = None):
    """Launch shape of later stream_extend calls on streams of ``ref`` (None:
    the process default); 0 = automatic."""
    _check(load_library().sdtw_stream_set_config(ref.handle if ref is not None else None,
                                                 int(strip), int(bands)))


def row_pool_trim():
    """Free the cached rows of closed streams on the current device."""
    _check(load_library().sdtw_row_pool_trim())


def row_budget_info():
    """(budget, in_use, cached) bytes on the current device."""
    b, u, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load_library().sdtw_row_budget_info(C.byref(b), C.byref(u), C.byref(c)))
    return b.value, u.value, c.value


class Stream:
    """One read extended chunk by chunk over a resident DP row."""

    def __init__(self, ref: Reference):
        h = C.c_void_p()
        _check(load_library().sdtw_stream_open(ref.handle, C.byref(h)))
        self._h = h
        self.ref = ref

    @property
    def handle(self):
        if self._h is None:
            raise SdtwError(5, "stream is closed")
        return self._h

    @property
    def closed(self) -> bool:
        return self._h is None

    @property
    def rows(self) -> int:
        r, n = C.c_int32(), C.c_int64()
        _check(load_library().sdtw_stream_info(self.handle, C.byref(r), C.byref(n)))
        return r.value

    def copy_row(self, out=None, stream=None):
        """The resident row gamma(rows, .) as an int32 / float32 device tensor."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.ref.n, dtype=torch.int32 if self.ref.dtype == I16
                              else torch.float32, device="cuda")
        _check(load_library().sdtw_stream_copy_row(self.handle, _dev(out), _stream(stream)))
        return out

    def close(self):
        if self._h is not None:
            _check(load_library().sdtw_stream_close(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_extend_wide(s, chunk, cols: int = 0, cost=None, end=None, stream=None):
    """sdtw_stream_extend_wide: extend one int16 stream by one chunk (device
    int16 tensor) over the whole device; returns (cost, end) device tensors."""
    torch = _torch()
    cost, end = _outputs(1, s.ref.dtype, chunk.device, cost, end)
    _check(load_library().sdtw_stream_extend_wide(
        s.handle, _dev(chunk, torch.int16, "chunk"), chunk.numel(), int(cols), _dev(cost),
        _dev(end, torch.int32, "end"), _stream(stream)))
    return cost, end


def stream_extend(streams, chunks, offsets, cost=None, end=None, stream=None):
    """sdtw_stream_extend: extend each stream by its chunk (CSR ``chunks`` on
    the device, host ``offsets``); returns (cost, end) device tensors."""
    torch = _torch()
    lib = load_library()
    ns = len(streams)
    if ns == 0:
        raise ValueError("no streams")
    offs = _offsets_host(offsets)
    if offs.size != ns + 1:
        raise ValueError("offsets must have len(streams) + 1 entries")
    dt = streams[0].ref.dtype
    qdt = torch.int16 if dt == I16 else torch.float32
    cost, end = _outputs(ns, dt, chunks.device, cost, end)
    handles = (C.c_void_p * ns)(*[s.handle for s in streams])
    _check(lib.sdtw_stream_extend(handles, ns, _dev(chunks, qdt, "chunks"),
                                  offs.ctypes.data_as(C.c_void_p), _dev(cost),
                                  _dev(end, torch.int32, "end"), _stream(stream)))
    return cost, end
