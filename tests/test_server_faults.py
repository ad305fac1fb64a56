"""Read Until server under injected faults, on the host with a simulated clock.

The serving loop (admission, continuous batching, decisions, fault handling)
runs unchanged; only its device side is replaced by a stand-in whose rows
hold the events they were extended by and whose results come from the
oracle on that prefix, ready a fixed simulated latency after submission.
Every result the server records is then checked against the oracle on the
pool read's true prefix (normalised with its first chunk), so a server that
sends a wrong segment (a restart that does not resend the prefix, a chunk
twice) fails.  Faults (section 2.2: a read must be decided while most of the
molecule is still in the pore; a late or lost decision only costs
sequencing time):

* a read that ends while its chunk is in flight (end_read): its result is
  ignored, its row released after the work, the channel moves on;
* a row closed elsewhere, between chunks and while a chunk is in flight
  (the library's close waits for the work): the read restarts on a new row
  from its first event, and its results stay exact;
* a chunk sent to a closed handle raises ESTATE in the binding;
* the row budget exhausted, also shrunk while serving, and in recompute
  mode: chunks queue for rows and every read is still served exactly;
* a chunk timeout: slow batches and long queues give reads up undecided.

The stand-in counts rows the server closes while work that uses them is in
flight (the real close would stall the loop): the server itself never does.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2211_07340_amd import binding as sd
from paper_2211_07340_amd import server as srv

E, MAX_EV, MIN_REJ = 50, 200, 100


class Clock:
    def __init__(self):
        self.t = 1000.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class Row:
    def __init__(self, dev, ti):
        self.dev, self.ti = dev, ti
        self.codes = np.zeros(0, np.int16)
        self.busy_until = -1.0
        self.closed = False
        self.closed_elsewhere = False

    def close(self):
        if self.closed:
            return
        if self.dev.clock() < self.busy_until and not self.closed_elsewhere:
            self.dev.closed_busy += 1
        self.closed = True
        self.dev.open -= 1


class Device:
    """Rows under a budget (a count of rows) and simulated batch latency."""
    def __init__(self, clock, refs, budget=None, latency=(0.01, 0.01)):
        self.clock, self.refs, self.budget, self.latency = clock, refs, budget, latency
        self.open = 0
        self.max_open = 0
        self.closed_busy = 0
        self.rows = []

    def open_row(self, ti):
        if self.budget is not None and self.open >= self.budget:
            raise sd.SdtwError(3, "row budget exhausted")
        self.open += 1
        self.max_open = max(self.max_open, self.open)
        r = Row(self, ti)
        self.rows.append(r)
        return r


class Tick(srv._Tick):
    pass


class FakeServer(srv.ReadUntilServer):
    def __init__(self, targets, cfg, device, clock, **kw):
        self.device = device
        self.seen = []  # (read, rows) of every result the server used
        super().__init__(targets, cfg, clock=clock, sleep=clock.sleep, **kw)

    def _decide(self, rd, cost, second=None):
        self.seen.append((rd, rd.rows))
        return super()._decide(rd, cost, second)

    def _setup_device(self):
        for t in self.targets:
            t.streams = list(range(max(1, self.cfg.streams_per_target)))

    def _prepare_run(self):
        if self.cfg.prewarm_rows and self.mode == "extend":
            self.prewarm()

    def _open_stream(self, ti):
        return self.device.open_row(ti)

    def _launch(self, ti, slot, batch):
        dev = self.device
        ready = self.clock() + dev.latency[ti]
        ref = dev.refs[ti]
        cost, end, c2, e2 = [], [], [], []
        cells = 0.0
        for _, rd, _, lo, hi in batch:
            seg = rd.raw[lo:hi]
            if rd.chunks_done == 0:
                rd.stats = oracle.zstats(seg)
            codes, _ = oracle.quantize(oracle.zapply(seg, *rd.stats), self.cfg.scale)
            row = rd.handle
            if row.closed:
                raise sd.SdtwError(5, "chunk sent to a closed row")
            if lo == 0:
                assert row.codes.size == 0, "a prefix sent to a row that already holds one"
            else:
                assert row.codes.size == lo, "a chunk that does not continue its row"
            row.codes = np.concatenate([row.codes, codes])
            row.busy_until = ready
            c, e, lr = oracle.sdtw_i64(row.codes, ref, lastrow=True)
            b = oracle.best_two(lr, self.cfg.mapq_window)
            cost.append(c)
            end.append(e)
            c2.append(np.iinfo(np.int32).max if b[3] < 0 else int(b[2]))
            e2.append(b[3])
            cells += seg.size * ref.size
        mq = self.cfg.decision == "mapq"
        return Tick(ready, ti, slot, [], np.array(cost), np.array(end),
                    np.array(c2) if mq else None, np.array(e2) if mq else None,
                    self.clock(), cells)

    def _tick_ready(self, tk):
        return self.clock() >= tk.event

    def _tick_results(self, tk):
        if self.clock() < tk.event:  # a blocking wait
            self.clock.t = tk.event
        return tk.cost, tk.end, tk.second, tk.second_end


@pytest.fixture(scope="module")
def world():
    table = synth.make_level_table()
    refs, pools = [], []
    for i, L in enumerate((1500, 2500)):
        genome = synth.make_genome(L, 300 + i)
        rd = synth.simulate_reads(genome, table, np.full(24, MAX_EV), 0.5, 71 + i)
        raws = [rd.values[rd.offsets[r]:rd.offsets[r + 1]] for r in range(24)]
        _, codes, _ = oracle.prepare_reference(genome, table, 6)
        refs.append(codes)
        pools.append((raws, np.asarray(rd.on_target, bool)))
    # tau: midpoint of the on- and off-target medians of the first chunk's
    # cost per event
    taus = []
    for (raws, on), ref in zip(pools, refs):
        s = []
        for raw in raws:
            m, v = oracle.zstats(raw[:E])
            q, _ = oracle.quantize(oracle.zapply(raw[:E], m, v), 64.0)
            s.append(oracle.sdtw_i64(q, ref)[0] / (64.0 * E))
        s = np.asarray(s)
        taus.append(0.5 * (np.median(s[on]) + np.median(s[~on])))
    return refs, pools, taus


def make(world, budget=None, latency=(0.01, 0.01), mode="extend", **cfg_kw):
    refs, pools, taus = world
    clock = Clock()
    dev = Device(clock, refs, budget, latency)
    targets = []
    for i, ((raws, on), ref) in enumerate(zip(pools, refs)):
        t = srv.Target(f"t{i}", None, raws, on)
        t.tau = taus[i]
        t.q_min = 30.0
        targets.append(t)
    kw = dict(channels=12, chunk_events=E, max_events=MAX_EV, min_reject_events=MIN_REJ,
              chunk_period_s=0.05, seed=5)
    kw.update(cfg_kw)
    rec = []
    server = FakeServer(targets, srv.ServerConfig(**kw), dev, clock, mode=mode, record=rec)
    return server, dev, clock, rec


def check_records(world, rec):
    """Every served result equals the oracle on the pool read's true prefix."""
    refs, pools, _ = world
    assert rec
    for t, pi, rows, cost, end, c2, e2 in rec:
        raw = pools[t][0][pi]
        m, v = oracle.zstats(raw[:E])
        q, _ = oracle.quantize(oracle.zapply(raw[:rows], m, v), 64.0)
        assert rows % E == 0 and E <= rows <= MAX_EV
        assert (cost, end) == oracle.sdtw_i64(q, refs[t]), (t, pi, rows)


def finish(dev):
    assert dev.open == 0, "rows left open after run()"
    assert dev.closed_busy == 0, "the server closed a row while its work was in flight"


def test_fault_free(world):
    server, dev, _, rec = make(world)
    res = server.run(2.0, 0.2)
    assert res["decisions"] > 20 and res["decision_accuracy"] > 0.8, res
    assert res["timeouts"] == res["ended"] == res["restarts"] == res["admission_waits"] == 0
    check_records(world, rec)
    finish(dev)


def _in_flight_channel(server):
    lp = server._loop
    for tk in lp.inflight:
        for c, rd, _, _ in tk.entries:
            if not rd.abandoned and lp.chan_read[c] is rd:
                return c, rd
    return None, None


def test_read_ends_while_its_chunk_is_in_flight(world):
    server, dev, clock, rec = make(world, latency=(0.03, 0.03))
    ended = []

    def end_one(s):
        c, rd = _in_flight_channel(s)
        if c is not None:
            s.end_read(c)
            assert rd.handle is not None  # released only after the work
            assert s._loop.chan_read[c] is not rd  # the channel moved on
            ended.append((rd, len(s.seen)))
    res = server.run(2.0, 0.1, events=[(0.3 + 0.2 * k, end_one) for k in range(8)])
    assert len(ended) >= 4 and res["ended"] == len(ended), res
    for rd, n in ended:
        assert rd.handle is None  # released when its batch was harvested
        assert not any(r is rd for r, _ in server.seen[n:])  # its late result unused
    assert res["decisions"] > 10
    check_records(world, rec)
    finish(dev)


def test_row_closed_elsewhere_restarts_exactly(world):
    server, dev, _, rec = make(world, latency=(0.02, 0.02))
    victims = []

    def lose(s, rd):
        # as the library does, the close waits for work in flight: a result
        # in flight stays valid
        rd.handle.closed_elsewhere = True
        rd.handle.close()
        victims.append((rd, rd.rows))

    def close_between_chunks(s):
        lp = s._loop
        for rd in lp.chan_read:
            if rd.handle is not None and rd.rows >= E and not s._in_flight(lp, rd):
                return lose(s, rd)

    def close_in_flight(s):
        c, rd = _in_flight_channel(s)
        if c is not None and rd.rows >= E:
            lose(s, rd)
    evs = [(0.25 + 0.15 * k, close_between_chunks if k % 2 else close_in_flight)
           for k in range(10)]
    res = server.run(2.0, 0.1, events=evs)
    assert len(victims) >= 4 and res["restarts"] >= 1, res
    # restarted reads were served past the rows they had when their row was
    # lost (the whole prefix resent to a new row; exact, checked below)
    again = [rd for rd, r0 in victims if any(r is rd and rows > r0 for r, rows in server.seen)]
    assert again, victims
    check_records(world, rec)
    finish(dev)


def test_chunk_to_closed_handle_raises_estate():
    s = sd.Stream.__new__(sd.Stream)
    s._h = None
    assert s.closed
    with pytest.raises(sd.SdtwError) as ei:
        s.handle
    assert ei.value.code == "ESTATE"


@pytest.mark.parametrize("mode", ["extend", "recompute"])
def test_row_budget_exhausted(world, mode):
    server, dev, _, rec = make(world, budget=4, mode=mode, channels=12)
    res = server.run(2.0, 0.1)
    assert res["admission_waits"] > 0 and res["max_waiting_chunks"] > 0, res
    assert dev.max_open <= 4
    assert res["decisions"] > 5, res
    check_records(world, rec)
    finish(dev)


def test_row_budget_shrinks_while_serving(world):
    server, dev, clock, rec = make(world, budget=12, channels=12, prewarm_rows=False)
    seen = {}

    def shrink(s):
        dev.budget = 3
        seen["open_at_shrink"] = dev.open

    def probe(s):
        seen["open_late"] = dev.open
    res = server.run(2.5, 0.1, events=[(0.8, shrink), (2.4, probe)])
    assert seen["open_at_shrink"] > 3 and seen["open_late"] <= 3, seen
    assert res["admission_waits"] > 0, res
    assert res["decisions"] > 5
    check_records(world, rec)
    finish(dev)


def test_chunk_timeout(world):
    # target 1's batches take 0.3 s against a 0.15 s timeout: its reads are
    # given up; target 0 is served as before
    server, dev, _, rec = make(world, latency=(0.01, 0.3), chunk_timeout_s=0.15)
    res = server.run(2.0, 0.1)
    assert res["timeouts"] > 0, res
    assert res["per_target"]["t0"]["decisions"] > 5
    assert res["per_target"]["t1"]["decisions"] == 0
    assert not any(r[0] == 1 for r in rec)  # no late result was used
    check_records(world, rec)
    finish(dev)


def test_chunk_timeout_of_queued_chunks(world):
    # two rows for twelve channels: chunks queue for rows longer than the
    # timeout and their reads are given up
    server, dev, _, rec = make(world, budget=2, chunk_timeout_s=0.05, prewarm_rows=False)
    res = server.run(2.0, 0.1)
    assert res["timeouts"] > 0 and res["admission_waits"] > 0, res
    assert res["decisions"] > 0
    check_records(world, rec)
    finish(dev)
