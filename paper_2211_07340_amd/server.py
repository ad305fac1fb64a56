"""Read Until serving loop over the streaming sDTW library.

Signal-level Read Until (section 2.2): every pore channel streams a read's
events; after each chunk the read is aligned against a target reference and
either kept, rejected (the pore voltage is reversed to eject it) or left to
sequence further.  A rejection is only useful while most of the molecule is
still unread, so decisions must come within a fraction of a second.

This module simulates the channels and runs the decisions through the C ABI:

* each channel emits a chunk of ``chunk_events`` events every
  ``chunk_period_s`` seconds of wall-clock time, from reads drawn from a
  pre-simulated pool per target (a channel starts its next read as soon as
  the current one is decided);
* a read's first chunk fixes its normalisation (sdtw_prepare_queries_ex
  returns the statistics, later chunks pass them back in), so that
  extending its resident row equals aligning the concatenated read;
* admission: a read gets a stream (a resident row) when the row budget
  allows; otherwise it waits, and its chunks queue;
* continuous batching: all chunks that have arrived (and whose read has no
  chunk in flight) are normalised and extended in one launch per target as
  soon as one of the target's HIP streams has no batch in flight; chunks
  that arrive meanwhile wait and join the next batch.  Targets have their
  own streams, so short-reference work never waits behind long-reference
  work (give the process at least as many hardware queues as streams,
  GPU_MAX_HW_QUEUES, or streams share queues and run in order);
* decision rules (readings; section 5.1 only says that a mapping quality
  is computed from the mapped positions and scores and that the selection
  criteria act on it):
  ``decision="cost"``: s = cost / (scale * rows), the mean per-event
  distance in z-units; keep if s <= tau, reject if rows >= ``max_events``
  or (rows >= ``min_reject_events`` and s > tau), else continue.
  ``decision="mapq"``: after each extension the library also returns the
  runner-up end farther than ``mapq_window`` columns from the best
  (sdtw_stream_best_two); q = ``mapq(best, second)``, a 0..60 score that
  grows with the relative gap between the two costs (a read that fits one
  locus much better than anywhere else is confidently placed); keep if
  q >= q_min, reject if rows >= ``max_events`` or (rows >=
  ``min_reject_events`` and q < q_min), else continue.
  tau and q_min are set per target as the midpoint of the medians of s (or
  q) of on-target and off-target reads' first chunks on a calibration set
  with its own seed.

``mode="recompute"`` aligns every chunk's whole prefix from scratch instead
(a fresh stream extended by the full prefix), for comparison.

Few chunks against a long reference.  A batched extension's time is that of
one chunk on its few waves (about 0.18 s for 400 events against 10 M
columns) however few chunks it holds, while sdtw_stream_extend_wide extends
one chunk over the whole device in a few milliseconds.  A batch of at most
``wide_chunks`` chunks (per target, by default the number whose whole-device
calls take no longer than one batched launch, measured at calibration) is
extended chunk by chunk over the whole device (``wide_chunks`` in the
report counts them); ``wide_burst_ms`` caps such a batch's duration, since
the whole device is its meanwhile and other targets' batches wait.  With
``wide_streams=2`` the chunks alternate between two HIP streams (one
chunk's look-back waits overlap the other's rows), which pays only where
the second stream has a hardware queue of its own: one shared with the
target's other stream serialises the two.

Faults.  A read must be decided while most of the molecule is still in the
pore (section 2.2); a lost or late decision only costs sequencing time, so
the loop gives such reads up rather than stalling:

* ``end_read(channel)``: the read ended before a decision (the molecule left
  the pore).  Its queued chunk is dropped, a chunk in flight finishes and its
  result is ignored, its row is released once no work that uses it is in
  flight (a close waits for such work), and the channel starts its next read;
* a row closed elsewhere (``handle.closed``): the read restarts on a new row
  from its first event -- the whole prefix in one extension, equal to
  extending it chunk by chunk;
* ``SDTW_EBUDGET`` on a row: the chunk waits for a row (admission queue); in
  recompute mode too, where each chunk takes a fresh row;
* ``chunk_timeout_s``: a read whose chunk has waited longer than this since it
  arrived, queued or in flight, is given up undecided (``timeouts``).

``run(..., events=[(seconds, fn), ...])`` calls ``fn(server)`` once the
server's clock passes each time, and the constructor takes the clock and the
wait of the loop, so that these faults can be forced on the host.

``ServerConfig(raw=True)`` serves raw current instead of events (targets from
``make_raw_targets``): every chunk period a channel's read has
``chunk_samples`` more samples (the pool's samples are resident on the
device, standing for the sequencer's signal buffer), and each batch first
cuts the new samples into events on the device (sdtw_detect_events_continue:
the detectors' state of every channel's read is kept on the device between
chunks, each sample is scanned once, events are delivered when later
samples cannot change them, the first ``trim_events`` dropped), appends them
to the channel's event buffer, then normalises and extends with the
buffered events not aligned yet.  A read's first extension waits for
``chunk_events`` events (its normalisation statistics); later ones take
whatever new events there are.  A read without new events waits for its
next chunk.
"""
from __future__ import annotations

import heapq
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as sd


WIDE_MAX_ROWS = 4096  # rows a stream may hold for sdtw_stream_extend_wide (SDTW_MAX_QUERY)


@dataclass
class ServerConfig:
    channels: int = 512
    chunk_events: int = 400
    chunk_period_s: float = 0.1
    max_events: int = 2000
    min_reject_events: int = 800
    scale: float = 64.0
    row_budget_bytes: int | None = None
    seed: int = 4004
    streams_per_target: int = 2        # HIP streams per target: launches of later ticks overlap
    stream_strip: int = 0              # sdtw_stream_set_config strip per target (0: the
                                       # library's choice by reference length)
    prewarm_rows: bool = True          # open (and close) rows for every channel before serving
    decision: str = "cost"             # "cost" or "mapq" (see the module doc)
    mapq_window: int = 2000            # columns around the best end excluded for the runner-up
    raw: bool = False                  # chunks of raw samples, events detected on the device
    chunk_samples: int = 2400          # raw mode: samples per channel per chunk period
    trim_events: int = 50              # raw mode: adaptor events dropped at a read's start
    chunk_timeout_s: float | None = None  # give up a read whose chunk waits longer (None: never)
    wide_chunks: int = -1              # batches of at most this many chunks extend chunk by
                                       # chunk over the whole device (int16 targets); -1: per
                                       # target at calibration, 0: never
    wide_burst_ms: float = 40.0        # calibration: at most this long per such batch (the
                                       # whole device is theirs meanwhile; other targets wait)
    wide_streams: int = 1              # HIP streams such a batch's chunks alternate over (1, 2;
                                       # 2 needs a hardware queue for the second, see above)


@dataclass
class Target:
    """A reference to align against, with a pool of simulated raw reads."""
    name: str
    ref: sd.Reference                  # int16 reference (prepared on the device)
    reads: list                        # raw pA event arrays (float32), >= max_events each
    on_target: np.ndarray              # bool per pool read
    tau: float = float("nan")          # cost threshold (z-units per event)
    q_min: float = float("nan")        # mapping-quality threshold (0..60)
    streams: list = field(default_factory=list)  # HIP streams of this target's work (set
                                                 # by the server that serves it)
    raw_dev: object = None             # raw mode: the pool's samples on the device
    raw_offs: object = None            # raw mode: int64 offsets of the pool's reads
    ev_states: object = None           # raw mode: detector state per channel (set by the server)
    ev_buf: object = None              # raw mode: [channels, max_events] detected events
    wide_max: int = 0                  # batches of at most this many chunks go over the whole
                                       # device (set by the serving config or calibration)
    wide_aux: object = None            # second HIP stream of those (set by the server)


@dataclass
class _Read:
    target: int
    pool_idx: int
    raw: np.ndarray
    start: float                       # time its first event was produced
    on: bool
    handle: object = None              # sd.Stream once admitted
    stats: object = None               # (1, 2) float64 device tensor after chunk 1
    rows: int = 0
    chunks_done: int = 0
    have: int = 0                      # raw mode: events detected (buffered) so far
    fresh_state: bool = True           # raw mode: its detector state is still to be reset
    restart: bool = False              # its row was lost: the next extension starts at event 0
    abandoned: str | None = None       # "ended" or "timeout" once given up undecided


@dataclass
class _Tick:
    event: object
    target: int
    slot: int                          # which of the target's streams
    entries: list                      # (channel, read, arrival, rows after)
    cost: object                       # pinned host copies of the results
    end: object
    second: object                     # pinned runner-up costs and ends ("mapq"), else None
    second_end: object
    t_submit: float
    cells: float


@dataclass
class ServerStats:
    decisions: int = 0
    kept: int = 0
    rejected: int = 0
    decided_on_target: int = 0
    kept_on_target: int = 0
    correct: int = 0
    decision_events: list = field(default_factory=list)
    chunks: int = 0
    cells: float = 0.0
    chunk_latency: list = field(default_factory=list)
    decision_latency: list = field(default_factory=list)
    decision_target: list = field(default_factory=list)
    admission_waits: int = 0
    max_queue: int = 0
    timeouts: int = 0                  # reads given up after a chunk timeout
    ended: int = 0                     # reads that ended before a decision (end_read)
    restarts: int = 0                  # reads restarted on a new row after theirs was lost
    wide_chunks: int = 0               # chunks extended over the whole device


def _median(x):
    return float(np.median(np.asarray(x))) if len(x) else float("nan")


_STREAMS: dict = {}  # device index -> HIP streams of this process, reused by every server


def _server_streams(torch, first: int, count: int) -> list:
    """Streams first .. first+count-1 of a per-device list that only grows.
    Servers and targets created later reuse them: a HIP stream created after
    GPU_MAX_HW_QUEUES others shares a hardware queue with an older one, and
    the work of streams on one queue runs in order, so fresh streams for
    every new server would serialise batches that should overlap."""
    pool = _STREAMS.setdefault(torch.cuda.current_device(), [])
    while len(pool) < first + count:
        pool.append(torch.cuda.Stream())
    return pool[first:first + count]


MAPQ_MAX = 60


def mapq(best, second):
    """Mapping-quality-like score from the best and runner-up alignment
    costs (non-negative; runner-up >= best): round(60 (second - best) /
    second), 0 when both are 0 (every locus fits perfectly: no information),
    60 when there is no runner-up (second = inf or the int32 maximum).
    Scale-free: the same for int16 codes and float32 values of one read."""
    b = np.asarray(best, dtype=np.float64)
    s = np.asarray(second, dtype=np.float64)
    none = ~np.isfinite(s) | (s >= np.iinfo(np.int32).max)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.where(s > 0, (s - b) / np.where(s > 0, s, 1.0), 0.0)
    q = np.floor(MAPQ_MAX * np.clip(g, 0.0, 1.0) + 0.5)
    return np.where(none, MAPQ_MAX, q).astype(np.int64)


@dataclass
class _Loop:
    """State of one run(): what every channel is doing."""
    chan_read: list                    # the read each channel is sequencing
    arrivals: list                     # heap of (arrival of a channel's next chunk, channel)
    waiting: list                      # (arrival, channel): chunks arrived, not submitted yet
    inflight: list                     # _Tick
    stats: ServerStats
    t0: float
    t_meas: float
    t_end: float
    host: dict = field(default_factory=dict)  # host time per loop phase: [total s, max s, calls]

    def in_window(self, now: float) -> bool:
        return self.t_meas <= now <= self.t_end


class ReadUntilServer:
    def __init__(self, targets: list[Target], cfg: ServerConfig | None = None,
                 mode: str = "extend", record: list | None = None, clock=None, sleep=None):
        """record: optional list receiving (target, pool read, rows, cost, end,
        second cost, second end) for every served chunk.  clock / sleep: the
        serving loop's time source and wait (time.perf_counter and time.sleep
        unless given; a host test passes a simulated clock)."""
        self.record = record
        self.targets = targets
        self.cfg = cfg or ServerConfig()
        if mode not in ("extend", "recompute"):
            raise ValueError("mode must be 'extend' or 'recompute'")
        if self.cfg.decision not in ("cost", "mapq"):
            raise ValueError("decision must be 'cost' or 'mapq'")
        if self.cfg.raw and (mode != "extend" or any(t.raw_dev is None for t in targets)):
            raise ValueError("raw mode extends resident rows of targets from make_raw_targets")
        self.mode = mode
        self.rng = np.random.default_rng(self.cfg.seed)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self._loop: _Loop | None = None
        self._setup_device()

    # ------------------------------------------------------------------
    # device side (the C ABI through the binding)
    def _setup_device(self):
        """HIP streams per target, the row budget, raw mode's detector states."""
        import torch
        self.torch = torch
        k = max(1, self.cfg.streams_per_target)
        for i, t in enumerate(self.targets):
            t.streams = _server_streams(torch, i * k, k)
        # one more per target: whole-device extensions of a batch alternate
        # between the batch's stream and this one, so that one chunk's
        # look-back waits overlap another chunk's rows
        for i, t in enumerate(self.targets):
            t.wide_aux = _server_streams(torch, len(self.targets) * k + i, 1)[0]
        if self.cfg.row_budget_bytes is not None:
            sd.set_row_budget(self.cfg.row_budget_bytes)
        if self.cfg.raw:
            for t in self.targets:
                t.ev_states = sd.EventStates(self.cfg.channels)
                t.ev_buf = torch.zeros((self.cfg.channels, self.cfg.max_events),
                                       dtype=torch.float32, device=torch.device("cuda"))

    def _prepare_run(self):
        for t in self.targets:
            sd.set_stream_config(self.cfg.stream_strip, 0, ref=t.ref)
        if self.cfg.prewarm_rows and self.mode == "extend":
            self.prewarm()

    def _open_stream(self, ti: int):
        """A resident row on target ti's reference (raises sd.SdtwError
        EBUDGET when the row budget is exhausted)."""
        return sd.Stream(self.targets[ti].ref)

    def _tick_ready(self, tk: _Tick) -> bool:
        return tk.event.query()

    def _tick_results(self, tk: _Tick):
        """(costs, ends, runner-up costs or None, runner-up ends or None)."""
        tk.event.synchronize()
        # pinned host copies, complete with the event
        return (tk.cost.numpy(), tk.end.numpy(),
                None if tk.second is None else tk.second.numpy(),
                None if tk.second_end is None else tk.second_end.numpy())

    # ------------------------------------------------------------------
    def calibrate(self, n_each: int = 128, seed: int = 77, group: int = 32):
        """Set each target's tau and q_min from the first chunks of reads of
        its pool drawn with another seed (aligned as one-chunk streams,
        ``group`` at a time, so the rows stay within a small budget)."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        M = self.cfg.chunk_events
        dev = torch.device("cuda")
        for t in self.targets:
            on_idx = np.nonzero(t.on_target)[0]
            off_idx = np.nonzero(~t.on_target)[0]
            pick = np.concatenate([rng.choice(on_idx, min(n_each, on_idx.size), replace=False),
                                   rng.choice(off_idx, min(n_each, off_idx.size), replace=False)])
            cost, second = [], []
            for g0 in range(0, pick.size, group):
                sub = pick[g0:g0 + group]
                offs = np.arange(sub.size + 1, dtype=np.int64) * M
                if self.cfg.raw:  # the first chunk_events events after the adaptor
                    rg = np.stack([t.raw_offs[sub], t.raw_offs[sub + 1]], 1).astype(np.int64)
                    fs = np.full(sub.size, self.cfg.trim_events, np.int32)
                    ev, cnt = sd.detect_events_prefix(
                        t.raw_dev, torch.from_numpy(rg).to(dev), torch.from_numpy(fs).to(dev),
                        self.cfg.trim_events, M)
                    if int(cnt.min().item()) < M:
                        raise ValueError("calibration reads have too few events")
                    raw_d = ev.reshape(-1)
                else:
                    raw_d = torch.from_numpy(
                        np.concatenate([t.reads[i][:M] for i in sub]).astype(np.float32)).to(dev)
                _, codes, _ = sd.prepare_queries(raw_d, torch.from_numpy(offs).to(dev),
                                                 self.cfg.scale)
                streams = [sd.Stream(t.ref) for _ in sub]
                try:
                    c, _ = sd.stream_extend(streams, codes, offs)
                    _, _, c2, _ = sd.stream_best_two(streams, self.cfg.mapq_window)
                    cost.append(c.cpu().numpy())
                    second.append(c2.cpu().numpy())
                finally:
                    torch.cuda.synchronize()
                    for st in streams:
                        st.close()
            cost = np.concatenate(cost).astype(np.float64)
            second = np.concatenate(second).astype(np.float64)
            on = t.on_target[pick]
            s = cost / (self.cfg.scale * M)
            q = mapq(cost, second)
            t.tau = 0.5 * (_median(s[on]) + _median(s[~on]))
            t.q_min = 0.5 * (_median(q[on]) + _median(q[~on]))
            t.wide_max = self._wide_max(t, raw_d[:M], dev)
        return {t.name: {"tau": t.tau, "q_min": t.q_min, "wide_max": t.wide_max}
                for t in self.targets}

    def _wide_max(self, t, chunk_raw, dev):
        """Chunks per batch up to which whole-device extensions (one per
        chunk, on ``wide_streams`` HIP streams) finish no later than one
        batched launch and within ``wide_burst_ms``: the configured number,
        or those times over the time per chunk, measured on two chunks of
        ``chunk_events`` rows (second chunks of two streams; best of two)."""
        if self.cfg.wide_chunks >= 0 or t.ref.dtype != sd.I16:
            return max(self.cfg.wide_chunks, 0) if t.ref.dtype == sd.I16 else 0
        torch = self.torch
        M = self.cfg.chunk_events
        sts = []
        try:
            for _ in range(2):
                sts.append(sd.Stream(t.ref))
        except sd.SdtwError as e:  # no room for two more rows: batched launches only
            for st in sts:
                st.close()
            if e.code == "EBUDGET":
                return 0
            raise
        offs = torch.tensor([0, M, 2 * M], dtype=torch.int64, device=dev)
        offs_np = np.array([0, M, 2 * M], np.int64)
        times = {"batch": [], "wide": []}
        main = torch.cuda.current_stream()
        aux = t.wide_aux if (t.wide_aux is not None and self.cfg.wide_streams > 1) else main
        try:
            _, codes, _ = sd.prepare_queries(torch.cat([chunk_raw, chunk_raw]), offs,
                                             self.cfg.scale)
            sd.stream_extend(sts, codes, offs_np)
            for way in ("batch", "wide") * 2:
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                if way == "batch":
                    sd.stream_extend(sts, codes, offs_np)
                else:
                    if aux is not main:
                        aux.wait_stream(main)
                    sd.stream_extend_wide(sts[0], codes[:M])
                    sd.stream_extend_wide(sts[1], codes[M:], stream=aux)
                    if aux is not main:
                        main.wait_stream(aux)
                b.record()
                b.synchronize()
                times[way].append(a.elapsed_time(b) / (1 if way == "batch" else 2))
        finally:
            torch.cuda.synchronize()
            for st in sts:
                st.close()
        budget = min(min(times["batch"]), self.cfg.wide_burst_ms)
        return int(budget // max(min(times["wide"]), 1e-3))

    # ------------------------------------------------------------------
    def _new_read(self, now: float) -> _Read:
        ti = int(self.rng.integers(0, len(self.targets)))
        t = self.targets[ti]
        pi = int(self.rng.integers(0, len(t.reads)))
        return _Read(ti, pi, t.reads[pi], now, bool(t.on_target[pi]))

    def _decide(self, rd: _Read, cost: float, second: float | None = None):
        """"keep", "reject" or None (sequence another chunk)."""
        t = self.targets[rd.target]
        if self.cfg.decision == "mapq":
            good = bool(mapq(cost, second) >= t.q_min)
        else:
            good = cost / (self.cfg.scale * rd.rows) <= t.tau
        if good:
            return "keep"
        if rd.rows >= self.cfg.max_events or rd.rows >= self.cfg.min_reject_events:
            return "reject"
        return None

    def prewarm(self):
        """Fill the library's row pool: open as many rows per target as there
        are channels (or as the budget allows) and close them again, so that
        admissions while serving reuse cached rows instead of allocating."""
        for ti in range(len(self.targets)):
            rows = []
            try:
                for _ in range(self.cfg.channels):
                    rows.append(self._open_stream(ti))
            except sd.SdtwError as e:
                if e.code != "EBUDGET":
                    raise
            for r in rows:
                r.close()

    # ------------------------------------------------------------------
    # faults and their handling
    def end_read(self, channel: int):
        """The sequencer reports that the read on ``channel`` ended before a
        decision (its molecule left the pore).  Its chunk still queued is
        dropped; a chunk in flight is left to finish and its result ignored;
        its row is released once no work that uses it is in flight (closing
        a row waits for such work, which would stall the serving loop); the
        channel starts its next read.  Only valid while run() serves (from
        one of its scheduled events)."""
        if self._loop is None:
            raise RuntimeError("end_read: the server is not serving")
        self._abandon(self._loop, channel, "ended", self.clock())

    def _in_flight(self, lp: _Loop, rd: _Read) -> bool:
        return any(e[1] is rd for tk in lp.inflight for e in tk.entries)

    def _release(self, rd: _Read):
        if rd.handle is not None:
            th = time.perf_counter()
            rd.handle.close()
            self._timed(self._loop, "stream_close", th)
            rd.handle = None

    def _abandon(self, lp: _Loop, c: int, why: str, now: float):
        """Give up the read on channel c (``why``: "ended" or "timeout")."""
        rd = lp.chan_read[c]
        rd.abandoned = why
        lp.waiting = [(a, ch) for a, ch in lp.waiting if ch != c]
        if any(ch == c for _, ch in lp.arrivals):
            lp.arrivals = [(a, ch) for a, ch in lp.arrivals if ch != c]
            heapq.heapify(lp.arrivals)
        if not self._in_flight(lp, rd):
            self._release(rd)
        if lp.in_window(now):
            if why == "timeout":
                lp.stats.timeouts += 1
            else:
                lp.stats.ended += 1
        lp.chan_read[c] = self._new_read(now)
        heapq.heappush(lp.arrivals, (now + self.cfg.chunk_period_s, c))

    def _expire(self, lp: _Loop, now: float):
        """Chunk timeout: a read whose chunk has waited (queued or in flight)
        longer than chunk_timeout_s since it arrived is given up undecided:
        a decision that late no longer saves sequencing time."""
        lim = self.cfg.chunk_timeout_s
        if lim is None:
            return
        late = [c for arr, c in lp.waiting if now - arr > lim]
        late += [c for tk in lp.inflight for c, rd, arr, _ in tk.entries
                 if not rd.abandoned and now - arr > lim]
        for c in late:
            self._abandon(lp, c, "timeout", now)

    @staticmethod
    def _timed(lp, key, t_start):
        if lp is None:
            return
        d = time.perf_counter() - t_start
        v = lp.host.setdefault(key, [0.0, 0.0, 0])
        v[0] += d
        v[1] = max(v[1], d)
        v[2] += 1

    # ------------------------------------------------------------------
    def run(self, duration_s: float, warmup_s: float = 0.0, events=None) -> dict:
        """Serve for warmup_s + duration_s seconds of the server's clock;
        report what was decided and measured during the last duration_s
        seconds.  events: optional (seconds after the start, callable taking
        the server) pairs, each called once when the clock passes its time
        (host-side fault injection: end_read, closing a row, the budget)."""
        cfg = self.cfg
        self._prepare_run()
        P = cfg.chunk_period_s
        t0 = self.clock()
        lp = _Loop([], [], [], [], ServerStats(), t0, t0 + warmup_s, t0 + warmup_s + duration_s)
        self._loop = lp
        pending = sorted(events or [], key=lambda e: e[0])
        for c in range(cfg.channels):
            start = t0 + float(self.rng.random()) * P
            lp.chan_read.append(self._new_read(start))
            heapq.heappush(lp.arrivals, (start + P, c))
        try:
            while True:
                now = self.clock()
                if now > lp.t_end:
                    break
                while pending and t0 + pending[0][0] <= now:
                    pending.pop(0)[1](self)
                self._harvest(lp)
                self._expire(lp, now)
                while lp.arrivals and lp.arrivals[0][0] <= now:
                    lp.waiting.append(heapq.heappop(lp.arrivals))
                lp.stats.max_queue = max(lp.stats.max_queue, len(lp.waiting))
                submitted = self._dispatch(lp)
                if not submitted:
                    nxt = lp.arrivals[0][0] if lp.arrivals else now + 0.002
                    self.sleep(max(0.0, min(nxt - self.clock(),
                                            0.0005 if lp.inflight else 0.002)))
            self._harvest(lp, block=True)
        finally:
            for tk in lp.inflight:  # only after an exception: wait before closing rows
                self._tick_results(tk)
            lp.inflight.clear()
            for rd in lp.chan_read:
                self._release(rd)
            self._loop = None
        return self._report(lp, duration_s)

    def _dispatch(self, lp: _Loop) -> bool:
        """Admit the waiting chunks' reads (a row each) and submit one batch
        per target that has a free HIP stream.  Returns whether anything was
        submitted."""
        cfg = self.cfg
        P = cfg.chunk_period_s
        groups: dict[int, list] = {}
        keep_waiting = []
        for arr, c in lp.waiting:
            rd = lp.chan_read[c]
            if rd.handle is not None and rd.handle.closed:
                # its row was closed elsewhere: the read restarts on a new row
                # from its first event (equal to extending it chunk by chunk)
                rd.handle = None
                rd.restart = rd.rows > 0
                lp.stats.restarts += 1
            if rd.handle is None:
                try:
                    th = time.perf_counter()
                    rd.handle = self._open_stream(rd.target)
                    self._timed(lp, "stream_open", th)
                except sd.SdtwError as e:
                    if e.code != "EBUDGET":
                        raise
                    lp.stats.admission_waits += 1
                    keep_waiting.append((arr, c))
                    continue
            groups.setdefault(rd.target, []).append((arr, c))
        # continuous batching: a target's ready chunks go out together on one
        # of its HIP streams that has no batch in flight; while all are busy
        # they wait and join the next batch
        submitted = False
        for ti, items in groups.items():
            if self._free_slot(ti, lp.inflight) is None:
                keep_waiting.extend(items)
                continue
            th = time.perf_counter()
            not_ready = self._submit(ti, items, lp.chan_read, lp.inflight)
            self._timed(lp, "submit " + self.targets[ti].name, th)
            submitted = True
            for _, c in not_ready:  # raw mode: no new final events yet
                rd = lp.chan_read[c]
                if rd.chunks_done * cfg.chunk_samples >= rd.raw.size + cfg.chunk_samples:
                    # the read is over without enough events: rejected
                    self._release(rd)
                    now = self.clock()
                    lp.chan_read[c] = self._new_read(now)
                    heapq.heappush(lp.arrivals, (now + P, c))
                else:
                    heapq.heappush(lp.arrivals, (rd.start + (rd.chunks_done + 1) * P, c))
        lp.waiting = keep_waiting
        return submitted

    def _harvest(self, lp: _Loop, block: bool = False):
        """Decide on the results of the batches that have completed."""
        P = self.cfg.chunk_period_s
        stats = lp.stats
        done = [tk for tk in lp.inflight if block or self._tick_ready(tk)]
        for tk in done:
            lp.inflight.remove(tk)
            th = time.perf_counter()
            costs, ends, seconds, second_ends = self._tick_results(tk)
            self._timed(lp, "results", th)
            now = self.clock()
            in_window = lp.in_window(now)
            if in_window:
                stats.cells += tk.cells
            for k, (c, rd, arr, rows) in enumerate(tk.entries):
                if self.mode == "recompute":
                    self._release(rd)  # a fresh row per chunk
                if rd.abandoned:
                    # ended or timed out while in flight: the result is not
                    # used and the row can be released now
                    self._release(rd)
                    continue
                if in_window:
                    stats.chunks += 1
                    stats.chunk_latency.append(now - arr)
                c2 = None if seconds is None else float(seconds[k])
                if self.record is not None:
                    self.record.append((rd.target, rd.pool_idx, rows, int(costs[k]),
                                        int(ends[k]), None if c2 is None else int(c2),
                                        None if second_ends is None else int(second_ends[k])))
                verdict = self._decide(rd, float(costs[k]), c2)
                if verdict is None:  # the read's next chunk
                    heapq.heappush(lp.arrivals, (rd.start + (rd.chunks_done + 1) * P, c))
                    continue
                if in_window:
                    stats.decisions += 1
                    stats.decision_latency.append(now - arr)
                    stats.decision_target.append(rd.target)
                    stats.kept += verdict == "keep"
                    stats.rejected += verdict == "reject"
                    stats.decided_on_target += rd.on
                    stats.kept_on_target += rd.on and verdict == "keep"
                    stats.decision_events.append(rd.rows)
                    stats.correct += (verdict == "keep") == rd.on
                self._release(rd)
                lp.chan_read[c] = self._new_read(now)
                heapq.heappush(lp.arrivals, (now + P, c))

    def _report(self, lp: _Loop, duration_s: float) -> dict:
        cfg = self.cfg
        stats = lp.stats
        lat = np.asarray(stats.decision_latency)
        clat = np.asarray(stats.chunk_latency)

        def pct(a, q):
            return round(float(np.percentile(a, q)) * 1e3, 2) if a.size else None

        return {
            "mode": self.mode,
            "seconds": round(duration_s, 2),
            "reads_per_s": round(stats.decisions / duration_s, 1),
            "decisions": stats.decisions,
            "kept": stats.kept,
            "rejected": stats.rejected,
            "decision": cfg.decision,
            "decision_accuracy": round(stats.correct / max(stats.decisions, 1), 4),
            "on_target_kept": round(stats.kept_on_target / max(stats.decided_on_target, 1), 4),
            "off_target_rejected": round(
                (stats.rejected - (stats.decided_on_target - stats.kept_on_target))
                / max(stats.decisions - stats.decided_on_target, 1), 4),
            "mean_events_at_decision": round(float(np.mean(stats.decision_events)), 1)
            if stats.decision_events else None,
            "chunks_per_s": round(stats.chunks / duration_s, 1),
            "gcups": round(stats.cells / duration_s / 1e9, 1),
            "decision_latency_p50_ms": pct(lat, 50),
            "decision_latency_p99_ms": pct(lat, 99),
            "chunk_latency_p50_ms": pct(clat, 50),
            "chunk_latency_p99_ms": pct(clat, 99),
            "admission_waits": stats.admission_waits,
            "max_waiting_chunks": stats.max_queue,
            "timeouts": stats.timeouts,
            "ended": stats.ended,
            "restarts": stats.restarts,
            "wide_chunks": stats.wide_chunks,
            "tau": {t.name: round(t.tau, 4) for t in self.targets},
            "q_min": {t.name: round(t.q_min, 2) for t in self.targets},
            "host_loop_ms": {k: {"total": round(v[0] * 1e3, 1), "max": round(v[1] * 1e3, 2),
                                 "calls": v[2]} for k, v in lp.host.items()},
            "per_target": {
                t.name: {"decisions": int((np.asarray(stats.decision_target) == ti).sum()),
                         "decision_latency_p50_ms": pct(lat[np.asarray(stats.decision_target)
                                                            == ti], 50),
                         "decision_latency_p99_ms": pct(lat[np.asarray(stats.decision_target)
                                                            == ti], 99)}
                for ti, t in enumerate(self.targets)},
        }

    def _extend(self, t, handles, codes, offs_np, hs):
        """Extend a batch's rows on HIP stream ``hs``: one batched launch, or
        for at most t.wide_max chunks one whole-device call per chunk (rows
        of at most WIDE_MAX_ROWS in all); (cost, end) device tensors."""
        lens = np.diff(offs_np)
        k = len(handles)
        if 1 <= k <= t.wide_max and all(h.rows + int(m) <= WIDE_MAX_ROWS
                                        for h, m in zip(handles, lens)):
            torch = self.torch
            cost = torch.empty(k, dtype=torch.int32, device=codes.device)
            end = torch.empty(k, dtype=torch.int32, device=codes.device)
            # chunks alternate between hs and the target's second stream,
            # which first waits for hs's work so far (the chunks' codes) and
            # which hs waits for at the end (the batch's results)
            aux = t.wide_aux if (k > 1 and t.wide_aux is not None and
                                 self.cfg.wide_streams > 1) else hs
            if aux is not hs:
                aux.wait_stream(hs)
            for i, h in enumerate(handles):
                sd.stream_extend_wide(h, codes[int(offs_np[i]):int(offs_np[i + 1])],
                                      cost=cost[i:i + 1], end=end[i:i + 1],
                                      stream=hs if i % 2 == 0 else aux)
            if aux is not hs:
                hs.wait_stream(aux)
            if self._loop is not None:
                self._loop.stats.wide_chunks += k
            return cost, end
        return sd.stream_extend(handles, codes, offs_np, stream=hs)

    def _free_slot(self, ti, inflight):
        """Index of one of target ti's HIP streams with no batch in flight."""
        busy = {tk.slot for tk in inflight if tk.target == ti}
        for k in range(len(self.targets[ti].streams)):
            if k not in busy:
                return k
        return None

    def _submit(self, ti, items, chan_read, inflight):
        """Normalise and extend the ready chunks of one target in one launch.
        Returns the reads that could not be extended yet (raw mode)."""
        if self.cfg.raw:
            return self._submit_raw(ti, items, chan_read, inflight)
        E = self.cfg.chunk_events
        # per chunk: (channel, read, arrival, first event, end event); the
        # read's whole prefix from scratch in recompute mode and after a
        # restart, else the new chunk alone
        batch = []
        for arr, c in items:
            rd = chan_read[c]
            lo = 0 if (self.mode == "recompute" or rd.restart) else rd.chunks_done * E
            batch.append((c, rd, arr, lo, (rd.chunks_done + 1) * E))
        slot = self._free_slot(ti, inflight)
        tk = self._launch(ti, slot, batch)
        for c, rd, arr, _, _ in batch:
            rd.chunks_done += 1
            rd.rows = rd.chunks_done * E
            rd.restart = False
            tk.entries.append((c, rd, arr, rd.rows))
        inflight.append(tk)
        return []

    def _launch(self, ti, slot, batch) -> _Tick:
        """Device work of one batch on target ti's HIP stream ``slot``: the
        raw events [lo, hi) of every read normalised (with its first chunk's
        statistics, computed here for a read's first chunk) and its row
        extended; results copied to pinned host memory behind an event."""
        torch = self.torch
        cfg = self.cfg
        t = self.targets[ti]
        dev = torch.device("cuda")
        hs = t.streams[slot]
        first = [b for b in batch if b[1].chunks_done == 0]
        cont = [b for b in batch if b[1].chunks_done > 0]
        code_parts, lens, order = [], [], []
        with torch.cuda.stream(hs):
            for group, fresh in ((first, True), (cont, False)):
                if not group:
                    continue
                segs = [rd.raw[lo:hi] for _, rd, _, lo, hi in group]
                # pinned staging and asynchronous copies: the host loop never
                # waits for earlier work queued on the stream
                offs_np = np.zeros(len(segs) + 1, np.int64)
                np.cumsum([x.size for x in segs], out=offs_np[1:])
                raw = torch.from_numpy(np.concatenate(segs).astype(np.float32)).pin_memory()
                offs = torch.from_numpy(offs_np).pin_memory()
                raw = raw.to(dev, non_blocking=True)
                offs = offs.to(dev, non_blocking=True)
                if fresh:
                    # the read's statistics are those of its first chunk
                    _, codes, _, st = sd.prepare_queries_ex(raw, offs, cfg.scale, stream=hs)
                    for k, (_, rd, _, _, _) in enumerate(group):
                        rd.stats = st[k:k + 1]
                else:
                    st_in = torch.cat([rd.stats for _, rd, _, _, _ in group])
                    _, codes, _, _ = sd.prepare_queries_ex(raw, offs, cfg.scale, st_in,
                                                           stream=hs)
                code_parts.append(codes)
                lens += [x.size for x in segs]
                order += group
            codes = torch.cat(code_parts) if len(code_parts) > 1 else code_parts[0]
            offs_np = np.zeros(len(lens) + 1, np.int64)
            np.cumsum(lens, out=offs_np[1:])
            handles = [rd.handle for _, rd, _, _, _ in order]
            cost, end = self._extend(t, handles, codes, offs_np, hs)
            pinned = [cost, end]
            if cfg.decision == "mapq":
                _, _, c2, e2 = sd.stream_best_two(handles, cfg.mapq_window, stream=hs)
                pinned += [c2, e2]
            # results to pinned host memory on the same stream: the event then
            # marks them readable and harvesting never issues a copy (a copy
            # to pageable memory could wait for other streams' work)
            host = []
            for x in pinned:
                h = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
                h.copy_(x, non_blocking=True)
                host.append(h)
            host += [None] * (4 - len(host))
            ev = torch.cuda.Event()
            ev.record(hs)
        # results follow `order` (first chunks, then continuing reads): put
        # the batch in that order so entries and results line up
        batch[:] = order
        return _Tick(ev, ti, slot, [], host[0], host[1], host[2], host[3], self.clock(),
                     float(sum(lens)) * t.ref.n)

    def _submit_raw(self, ti, items, chan_read, inflight):
        """Raw mode: events of each read's new samples (the detectors
        continue from their state), buffered per channel, then the same
        normalisation and extension as for event chunks."""
        torch = self.torch
        cfg = self.cfg
        dev = torch.device("cuda")
        t = self.targets[ti]
        E = cfg.chunk_events
        keep = 2 * E
        slot = self._free_slot(ti, inflight)
        hs = t.streams[slot]
        n = len(items)
        rg = np.empty((n, 2), np.int64)
        chans = np.array([c for _, c in items], np.int32)
        new = [c for _, c in items if chan_read[c].fresh_state]
        for k, (_, c) in enumerate(items):
            rd = chan_read[c]
            a, b = int(t.raw_offs[rd.pool_idx]), int(t.raw_offs[rd.pool_idx + 1])
            rg[k] = (a, min(b, a + (rd.chunks_done + 1) * cfg.chunk_samples))
        waiting = []
        with torch.cuda.stream(hs):
            if new:
                t.ev_states.reset(torch.from_numpy(np.array(new, np.int32)).to(
                    dev, non_blocking=True), stream=hs)
                for c in new:
                    chan_read[c].fresh_state = False
            rg_d = torch.from_numpy(rg).pin_memory().to(dev, non_blocking=True)
            ch_d = torch.from_numpy(chans).pin_memory().to(dev, non_blocking=True)
            ev, cnt = t.ev_states.detect(t.raw_dev, rg_d, ch_d, cfg.trim_events, keep,
                                         stream=hs)
            cnt_h = torch.empty(n, dtype=torch.int32, pin_memory=True)
            cnt_h.copy_(cnt, non_blocking=True)
            hs.synchronize()  # this stream had no batch in flight: only the detection
            cnt_np = cnt_h.numpy().copy()
            if (cnt_np < 0).any():
                raise RuntimeError("event detection: more boundaries waiting than it keeps")
            # append the new events to the channels' buffers
            have = np.array([chan_read[c].have for _, c in items], np.int64)
            add = np.minimum(cnt_np, cfg.max_events - have)
            if add.any():
                j = torch.arange(keep, device=dev)[None, :]
                mask = j < torch.from_numpy(add).to(dev)[:, None]
                rows_i = ch_d.long()[:, None].expand(n, keep)[mask]
                cols_i = (torch.from_numpy(have).to(dev)[:, None] + j)[mask]
                t.ev_buf[rows_i, cols_i] = ev[mask]
            # a read's events not aligned yet start at `base` (0 after a
            # restart: the whole buffered prefix again, on a new row)
            base = np.array([0 if chan_read[c].restart else chan_read[c].rows for _, c in items],
                            np.int64)
            take = np.zeros(n, np.int64)
            for k, (_, c) in enumerate(items):
                rd = chan_read[c]
                rd.have += int(add[k])
                avail = rd.have - base[k]
                if rd.rows == 0:
                    take[k] = E if avail >= E else 0  # the first chunk fixes the statistics
                else:
                    take[k] = avail
            entries, code_parts, lens = [], [], []
            for fresh in (True, False):
                sel = [k for k, (_, c) in enumerate(items)
                       if take[k] > 0 and (chan_read[c].rows == 0) == fresh]
                if not sel:
                    continue
                group = [items[k] for k in sel]
                tk = np.array([take[k] for k in sel], np.int64)
                start = base[sel]
                width = int(tk.max())
                j = torch.arange(width, device=dev)[None, :]
                mask = j < torch.from_numpy(tk).to(dev)[:, None]
                rows_i = torch.from_numpy(chans[sel].astype(np.int64)).to(dev)[:, None] \
                    .expand(len(sel), width)[mask]
                cols_i = (torch.from_numpy(start).to(dev)[:, None] + j)[mask]
                vals = t.ev_buf[rows_i, cols_i]  # the taken events, read after read
                offs_np = np.zeros(len(sel) + 1, np.int64)
                np.cumsum(tk, out=offs_np[1:])
                offs = torch.from_numpy(offs_np).to(dev, non_blocking=True)
                if fresh:
                    _, codes, _, st = sd.prepare_queries_ex(vals, offs, cfg.scale, stream=hs)
                    for i2, (_, c) in enumerate(group):
                        chan_read[c].stats = st[i2:i2 + 1]
                else:
                    st_in = torch.cat([chan_read[c].stats for _, c in group])
                    _, codes, _, _ = sd.prepare_queries_ex(vals, offs, cfg.scale, st_in,
                                                           stream=hs)
                code_parts.append(codes)
                lens += tk.tolist()
                entries += [(c, chan_read[c], arr, int(take[k])) for k, (arr, c) in
                            zip(sel, group)]
            for k, (arr, c) in enumerate(items):
                if take[k] == 0:
                    waiting.append((arr, c))
            if not entries:
                for _, c in waiting:
                    chan_read[c].chunks_done += 1
                return waiting
            codes = torch.cat(code_parts) if len(code_parts) > 1 else code_parts[0]
            offs_np = np.zeros(len(lens) + 1, np.int64)
            np.cumsum(lens, out=offs_np[1:])
            handles = [rd.handle for _, rd, _, _ in entries]
            cost, end = self._extend(t, handles, codes, offs_np, hs)
            pinned = [cost, end]
            if cfg.decision == "mapq":
                _, _, c2, e2 = sd.stream_best_two(handles, cfg.mapq_window, stream=hs)
                pinned += [c2, e2]
            host = []
            for x in pinned:
                h = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
                h.copy_(x, non_blocking=True)
                host.append(h)
            host += [None] * (4 - len(host))
            evt = torch.cuda.Event()
            evt.record(hs)
        out = []
        for c, rd, arr, tk in entries:
            rd.chunks_done += 1
            rd.rows = (0 if rd.restart else rd.rows) + tk
            rd.restart = False
            out.append((c, rd, arr, rd.rows))
        for _, c in waiting:
            chan_read[c].chunks_done += 1
        inflight.append(_Tick(evt, ti, slot, out, host[0], host[1], host[2], host[3],
                              self.clock(), float(sum(lens)) * t.ref.n))
        return waiting


def make_raw_targets(specs, torch_device, k: int = 6, scale: float = 64.0):
    """Raw-mode targets from (name, genome uint8 array, level table, raw
    samples float32 (reads concatenated), int64 offsets, on-target flags):
    the reference is prepared on the device and the pool's samples are
    uploaded once."""
    torch = __import__("torch")
    out = []
    for name, genome, table, values, offsets, on in specs:
        g = torch.from_numpy(genome).to(torch_device)
        t = torch.from_numpy(table).to(torch_device)
        _, codes, _ = sd.prepare_reference(g, t, k, scale)
        offs = np.asarray(offsets, np.int64)
        reads = [values[offs[r]:offs[r + 1]] for r in range(offs.size - 1)]
        tg = Target(name, sd.Reference(codes), reads, np.asarray(on, bool))
        tg.raw_dev = torch.from_numpy(np.ascontiguousarray(values, np.float32)).to(torch_device)
        tg.raw_offs = offs
        out.append(tg)
    return out


def make_targets(specs, torch_device, k: int = 6, scale: float = 64.0):
    """Targets from (name, genome uint8 array, level table, read pool raw
    arrays, on-target flags) tuples: the reference is prepared on the device
    (sdtw_prepare_reference) and loaded as int16."""
    torch = __import__("torch")
    out = []
    for name, genome, table, reads, on in specs:
        g = torch.from_numpy(genome).to(torch_device)
        t = torch.from_numpy(table).to(torch_device)
        _, codes, _ = sd.prepare_reference(g, t, k, scale)
        out.append(Target(name, sd.Reference(codes), reads, np.asarray(on, bool)))
    return out
