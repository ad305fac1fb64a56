"""Event detection on the device (sdtw_detect_events) against the oracle,
value for value (float32 equality): simulated raw reads of on-target,
background-genome and noise reads, several (trim, keep) pairs including
reads with fewer events than asked for, reads shorter than the t-test
windows, empty reads, and noise-free steps; then the whole pre-processing
chain (raw -> events -> normalisation -> alignment) against the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import events as ev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.load_library()
    return torch.device("cuda:0")


def gpu_events(dev, values, offsets, trim, keep):
    e, c = sd.detect_events(torch.from_numpy(np.asarray(values, np.float32)).to(dev),
                            torch.from_numpy(np.asarray(offsets, np.int64)).to(dev), trim, keep)
    torch.cuda.synchronize()
    return e.cpu().numpy(), c.cpu().numpy()


def check(values, offsets, e, c, trim, keep):
    for r in range(len(offsets) - 1):
        want = ev.query_events(values[offsets[r]:offsets[r + 1]], trim, keep)
        assert c[r] == want.size, (r, c[r], want.size)
        assert np.array_equal(e[r, :c[r]], want), r
        assert not e[r, c[r]:].any()


@pytest.mark.parametrize("trim,keep", [(50, 250), (0, 1), (0, 33), (7, 400), (300, 20),
                                       (0, 4096)])
def test_simulated_reads_match_oracle(dev, trim, keep):
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    bg = synth.make_genome(200_000, 77)
    raw = synth.simulate_raw(g, synth.make_level_table(), 12, 240, 0.5, trim + keep,
                             off_genome=bg)
    note(f"events trim={trim} keep={keep} samples={raw.values.size}")
    e, c = gpu_events(dev, raw.values, raw.offsets, trim, keep)
    check(raw.values, raw.offsets, e, c, trim, keep)


def test_noise_reads_and_edge_lengths(dev):
    rng = np.random.default_rng(8)
    parts = [rng.normal(90, 12, size=n).astype(np.float32)
             for n in (0, 1, 2, 5, 6, 7, 12, 13, 511, 512, 513, 1025, 3000)]
    values, offsets = synth.csr(parts)
    for trim, keep in ((0, 5), (3, 50), (0, 4096)):
        note(f"events edge lengths trim={trim} keep={keep}")
        e, c = gpu_events(dev, values, offsets, trim, keep)
        check(values, offsets, e, c, trim, keep)


@pytest.mark.parametrize("nreads", [4096, 8192])
def test_large_batches_share_waves(dev, nreads):
    # batches large enough that two or four reads share a wave: a sample of
    # reads in every position within a wave against the oracle
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), nreads, 60, 0.5, nreads, adaptor=8)
    note(f"events {nreads} reads, {raw.values.size} samples")
    e, c = gpu_events(dev, raw.values, raw.offsets, 10, 60)
    rng = np.random.default_rng(nreads)
    pick = sorted(set(rng.choice(nreads, 20, replace=False).tolist() + [0, 1, 2, 3, nreads - 1]))
    for r in pick:
        want = ev.query_events(raw.values[raw.offsets[r]:raw.offsets[r + 1]], 10, 60)
        assert c[r] == want.size, r
        assert np.array_equal(e[r, :c[r]], want), r
        assert not e[r, c[r]:].any()


def test_prefixes_of_reads_being_received(dev):
    # the events written for a prefix are the whole read's, from `first` on
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 10, 300, 0.5, 404)
    rng = np.random.default_rng(5)
    ranges, firsts, whole = [], [], []
    for r in range(raw.nreads):
        a, b = int(raw.offsets[r]), int(raw.offsets[r + 1])
        full = ev.events(raw.values[a:b])
        for L in (0, 4, 5, 6, 7, 40, int(rng.integers(100, b - a)), b - a):
            ranges.append((a, a + L))
            firsts.append(int(rng.integers(0, 60)))
            whole.append(full)
    ranges.append((0, 100))  # a first event beyond max_first: count -1
    firsts.append(61)
    note(f"prefix events: {len(firsts)} prefixes")
    rg = torch.tensor(ranges, dtype=torch.int64, device=dev)
    fs = torch.tensor(firsts, dtype=torch.int32, device=dev)
    x = torch.from_numpy(raw.values).to(dev)
    e, c = sd.detect_events_prefix(x, rg, fs, 60, 300)
    torch.cuda.synchronize()
    e, c = e.cpu().numpy(), c.cpu().numpy()
    for i, full in enumerate(whole):
        f, n = firsts[i], int(c[i])
        assert 0 <= n <= 300
        assert np.array_equal(e[i, :n], full[f:f + n]), (i, ranges[i], f, n)
        assert not e[i, n:].any()
        if ranges[i][1] - ranges[i][0] < 6:
            assert n == 0
    assert c[-1] == -1 and not e[-1].any()


def test_continuing_detection_over_chunks(dev):
    # reads received in chunks of different sizes, each sample scanned once:
    # the events delivered call after call are the whole read's
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 6, 500, 0.5, 606)
    x = torch.from_numpy(raw.values).to(dev)
    n = raw.nreads
    states = sd.EventStates(n + 3)
    slots = torch.tensor([n + 2 - r for r in range(n)], dtype=torch.int32, device=dev)
    states.reset(slots)
    chunk = [300, 700, 1200, 2400, 2400, 5000]
    got = [[] for _ in range(n)]
    lens = np.zeros(n, np.int64)
    total = np.diff(raw.offsets)
    for call in range(40):
        lens = np.minimum(total, lens + np.array(chunk))
        rg = np.stack([raw.offsets[:-1], raw.offsets[:-1] + lens], 1).astype(np.int64)
        e, c = states.detect(x, torch.from_numpy(rg).to(dev), slots, 50, 1200)
        torch.cuda.synchronize()
        e, c = e.cpu().numpy(), c.cpu().numpy()
        assert (c >= 0).all(), c
        for r in range(n):
            got[r].append(e[r, :c[r]].copy())
            assert not e[r, c[r]:].any()
        if (lens == total).all() and call > 0 and not c.any():
            break
    note(f"continuing detection: {call + 1} calls")
    for r in range(n):
        full = ev.events(raw.values[raw.offsets[r]:raw.offsets[r + 1]])
        mine = np.concatenate(got[r])
        assert np.array_equal(mine, full[50:50 + mine.size]), r
        assert mine.size >= full.size - 50 - 3, (r, mine.size, full.size)


def test_continuing_detection_overflow_is_reported(dev):
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 1, 300, 1.0, 3)
    x = torch.from_numpy(raw.values).to(dev)
    states = sd.EventStates(1)
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    states.reset(slots)
    rg = torch.tensor([[0, int(raw.offsets[1])]], dtype=torch.int64, device=dev)
    _, c = states.detect(x, rg, slots, 0, 1)  # one event may leave per call
    torch.cuda.synchronize()
    assert int(c.item()) == -1


def test_noise_free_steps(dev):
    rng = np.random.default_rng(9)
    lens = rng.integers(3, 16, size=400)
    lv = rng.normal(90, 12, size=400).astype(np.float32)
    x = np.repeat(lv, lens)
    e, c = gpu_events(dev, x, [0, x.size], 10, 300)
    assert c[0] == 300 and np.array_equal(e[0], lv[10:310])


def test_raw_to_alignment_chain(dev):
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    table = synth.make_level_table()
    raw = synth.simulate_raw(g, table, 16, 320, 0.5, 61)
    _, ref, _ = oracle.prepare_reference(g, table, synth.K)
    e, c = gpu_events(dev, raw.values, raw.offsets, 50, 250)
    assert (c == 250).all()
    ev_offs = np.arange(17, dtype=np.int64) * 250
    _, q, _ = sd.prepare_queries(torch.from_numpy(e.reshape(-1)).to(dev),
                                 torch.from_numpy(ev_offs).to(dev), 64.0)
    r = sd.Reference(torch.from_numpy(ref).to(dev))
    plan = sd.Plan(ev_offs, sd.I16)
    cost, end = sd.align_batch(r, plan, q)
    torch.cuda.synchronize()
    # the oracle's chain on the same raw samples
    qs = [oracle.quantize(oracle.znorm(ev.query_events(
        raw.values[raw.offsets[i]:raw.offsets[i + 1]], 50, 250)), 64.0)[0] for i in range(16)]
    qo, offs = synth.csr(qs)
    wc, we, _ = oracle.batch(oracle.I64, qo, offs, ref)
    assert cost.cpu().numpy().tolist() == wc.astype(np.int64).tolist()
    assert end.cpu().numpy().tolist() == we.tolist()
    plan.close()
    r.close()
