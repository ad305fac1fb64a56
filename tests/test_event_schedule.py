"""CPU model of the event-detection kernel's control flow (k_detect_events),
checked against the oracle: positions in blocks (512, or 128 when a wave
serves four reads), boundaries inserted
into a sorted list that keeps only the trim + keep smallest, the early stop
once those are final (below every open candidate), and the event sums from
the list.  The t statistics are the oracle's; what is tested is that
stopping early and truncating the list never change the events returned.
No GPU.
"""
import math

import numpy as np
import pytest

import synth
from oracle import events as ev

def kernel_model(x, trim, keep, BLOCK=512, prefix=False):
    """prefix: x is the start of a longer read (scan to L - 5, final events
    only)."""
    ts, tl = ev.tstat(x, 3), ev.tstat(x, 6)
    L, cap = x.size, trim + keep
    scan = max(L - 5, 0) if prefix else L
    det = {k: dict(masked_to=-1, peak_pos=-1, peak_val=math.inf, valid=False)
           for k in ("s", "l")}
    bs = []

    def insert(b):
        if len(bs) == cap and b >= bs[-1]:
            return
        if b in bs:
            return
        bs.append(b)
        bs.sort()
        del bs[cap:]

    def step(k, w, thr, i, v):
        d = det[k]
        if d["masked_to"] >= i:
            return
        if d["peak_pos"] < 0:
            if v < d["peak_val"]:
                d["peak_val"] = v
            elif v - d["peak_val"] > ev.PEAK_HEIGHT:
                d["peak_val"], d["peak_pos"] = v, i
            return
        if v > d["peak_val"]:
            d["peak_val"], d["peak_pos"] = v, i
        if k == "s" and d["peak_val"] > thr:
            det["l"].update(masked_to=d["peak_pos"] + 6, peak_pos=-1, peak_val=math.inf,
                            valid=False)
        if d["peak_val"] - v > ev.PEAK_HEIGHT and d["peak_val"] > thr:
            d["valid"] = True
        if d["valid"] and i - d["peak_pos"] > w // 2:
            insert(d["peak_pos"])
            d.update(peak_pos=-1, peak_val=v, valid=False)

    stopped = False
    cut = 0
    for b0 in range(0, scan, BLOCK):
        end = min(scan, b0 + BLOCK)
        for i in range(b0, end):
            step("s", 3, ev.T_SHORT, i, ts[i])
            step("l", 6, ev.T_LONG, i, tl[i])
        cut = end
        for k in ("s", "l"):
            if 0 <= det[k]["peak_pos"] < cut:
                cut = det[k]["peak_pos"]
        if len(bs) == cap and bs[-1] < cut:
            stopped = True
            break
    if stopped:
        closed = cap
    elif prefix:  # events whose end boundary is final
        closed = sum(1 for b in bs if b < cut)
    else:
        closed = len(bs) + 1 if L > 0 else 0
    n_out = max(min(closed, cap) - trim, 0)
    out = []
    for k in range(n_out):
        j = trim + k
        lo = 0 if j == 0 else bs[j - 1]
        up = bs[j] if j < len(bs) else L
        s = 0.0
        for q in range(lo, up):
            s += float(x[q])
        out.append(s / (up - lo))
    return np.asarray(out, np.float64).astype(np.float32), stopped


@pytest.mark.parametrize("block", [128, 512])
@pytest.mark.parametrize("trim,keep", [(0, 1), (0, 7), (5, 20), (50, 250), (50, 600),
                                       (400, 30), (0, 4000)])
def test_model_equals_oracle(trim, keep, block):
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 5, 300, 0.6, trim * 7 + keep)
    stops = 0
    for r in range(raw.nreads):
        x = raw.values[raw.offsets[r]:raw.offsets[r + 1]]
        got, stopped = kernel_model(x, trim, keep, block)
        want = ev.query_events(x, trim, keep)
        assert np.array_equal(got, want), (r, trim, keep)
        stops += stopped
    if trim + keep <= 300:  # reads have ~550 events: most stop early
        assert stops >= 4


def test_reads_shorter_than_windows():
    for L in (0, 1, 2, 5, 6, 7, 12):
        x = np.linspace(80, 100, L).astype(np.float32)
        got, _ = kernel_model(x, 0, 5)
        assert np.array_equal(got, ev.query_events(x, 0, 5))


@pytest.mark.parametrize("first,keep", [(0, 400), (50, 250), (130, 40), (0, 6000)])
def test_prefix_events_are_those_of_the_whole_read(first, keep):
    # a read still arriving: the events written for any prefix are the whole
    # read's events from `first` on, as many as are final
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 3, 300, 0.6, first + keep)
    rng = np.random.default_rng(first)
    for r in range(raw.nreads):
        x = raw.values[raw.offsets[r]:raw.offsets[r + 1]]
        full = ev.events(x)
        for L in sorted(set(rng.integers(0, x.size + 1, size=6).tolist() + [0, 3, x.size])):
            got, _ = kernel_model(x[:L], first, keep, 128, prefix=True)
            assert np.array_equal(got, full[first:first + got.size]), (r, L)
        # with the whole read given, only the last event or two stay open
        got, _ = kernel_model(x, first, keep, 128, prefix=True)
        assert got.size >= min(keep, max(full.size - first - 3, 0))


class ContinuingModel:
    """The continuing kernel (k_events_continue) on the CPU: the detectors'
    state and up to 32 pending boundaries kept between calls."""

    PEND = 32

    def __init__(self):
        self.pos, self.last, self.index = 0, 0, 0
        self.det = {k: dict(masked_to=-1, peak_pos=-1, peak_val=math.inf, valid=False)
                    for k in ("s", "l")}
        self.pend = []
        self.overflow = False

    def call(self, x, trim, keep):
        L = x.size
        scan = max(L - 5, 0)
        ts, tl = ev.tstat(x, 3), ev.tstat(x, 6)

        def step(k, w, thr, i, v):
            d = self.det[k]
            if d["masked_to"] >= i:
                return
            if d["peak_pos"] < 0:
                if v < d["peak_val"]:
                    d["peak_val"] = v
                elif v - d["peak_val"] > ev.PEAK_HEIGHT:
                    d["peak_val"], d["peak_pos"] = v, i
                return
            if v > d["peak_val"]:
                d["peak_val"], d["peak_pos"] = v, i
            if k == "s" and d["peak_val"] > thr:
                self.det["l"].update(masked_to=d["peak_pos"] + 6, peak_pos=-1,
                                     peak_val=math.inf, valid=False)
            if d["peak_val"] - v > ev.PEAK_HEIGHT and d["peak_val"] > thr:
                d["valid"] = True
            if d["valid"] and i - d["peak_pos"] > w // 2:
                b = d["peak_pos"]
                if b not in self.pend:
                    if len(self.pend) == self.room:
                        self.overflow = True
                    else:
                        self.pend = sorted(self.pend + [b])
                d.update(peak_pos=-1, peak_val=v, valid=False)

        self.room = keep + self.PEND  # the pending list's room during a call
        for i in range(self.pos, scan):
            step("s", 3, ev.T_SHORT, i, ts[i])
            step("l", 6, ev.T_LONG, i, tl[i])
        self.pos = max(self.pos, scan)
        cut = self.pos
        for k in ("s", "l"):
            if 0 <= self.det[k]["peak_pos"] < cut:
                cut = self.det[k]["peak_pos"]
        out = []
        while self.pend and self.pend[0] < cut and len(out) < keep:
            b = self.pend.pop(0)
            if self.index >= trim:
                out.append(float(np.mean(x[self.last:b].astype(np.float64))))
            self.last, self.index = b, self.index + 1
        if len(self.pend) > self.PEND:  # more than 32 carried to the next call
            self.overflow = True
        return np.asarray(out, np.float32)


@pytest.mark.parametrize("trim,keep,chunk", [(50, 800, 2400), (0, 800, 1000), (7, 64, 300)])
def test_continuing_detector_delivers_the_whole_read_events(trim, keep, chunk):
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 3, 400, 0.6, chunk)
    for r in range(raw.nreads):
        x = raw.values[raw.offsets[r]:raw.offsets[r + 1]]
        full = ev.events(x)
        m = ContinuingModel()
        got = []
        for n in list(range(chunk, x.size, chunk)) + [x.size, x.size]:
            got.append(m.call(x[:n], trim, keep))
            assert not m.overflow
        got = np.concatenate(got)
        want = full[trim:trim + got.size]
        # np.mean sums pairwise, the kernel in index order: compare closely
        assert np.allclose(got, want, rtol=1e-6, atol=0), r
        assert got.size >= full.size - trim - 3  # all but the last open events


def test_continuing_detector_overflows_loudly():
    # more than 32 boundaries left after a call that may write only one
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 1, 200, 1.0, 3)
    x = raw.values[raw.offsets[0]:raw.offsets[1]]
    m = ContinuingModel()
    m.call(x, 0, 1)
    assert m.overflow
