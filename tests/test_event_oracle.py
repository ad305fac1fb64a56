"""Pins of the event-detection oracle (oracle.events) against what the
detector's definition fixes: the t statistic's closed form, hand-worked peak
detector runs (threshold, peak height, emission delay, masking of the long
detector), exact recovery of noise-free steps, partition invariants, and,
end to end, that events of simulated raw reads align where the read came
from.  No GPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import events as ev


def test_tstat_closed_form():
    x = np.array([1, 2, 3, 4, 5, 6], np.float32)
    t = ev.tstat(x, 3)
    # m1 = 2, m2 = 5, v1 = v2 = 2/3: 3 / sqrt(4/9) = 4.5
    assert t[3] == pytest.approx(4.5, rel=1e-15)
    assert t[0] == t[1] == t[2] == t[4] == t[5] == 0.0  # outside 3 <= i <= 3
    assert not ev.tstat(np.full(40, 7.5, np.float32), 6).any()
    # a step between constant windows: the variance floor, not a division by 0
    step = np.array([10, 10, 10, 12, 12, 12], np.float32)
    assert ev.tstat(step, 3)[3] == pytest.approx(2.0 / ev.DEN_FLOOR)
    # symmetric in the sign of the step, and shift invariant
    assert ev.tstat(step[::-1].copy(), 3)[3] == ev.tstat(step, 3)[3]
    y = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float32)
    assert np.allclose(ev.tstat(y + 100, 3), ev.tstat(y, 3), rtol=1e-9)


def _t(vals, n=16):
    t = np.zeros(n)
    for i, v in vals.items():
        t[i] = v
    return t


def test_peak_detector_hand_worked():
    # short detector: a candidate opens at 2 (0.5 > 0 + 0.2), moves to 3
    # (2.0), becomes valid at 4 (2.0 - 1.0 > 0.2, 2.0 > 1.4) and is emitted at
    # 5, the first position more than 3 // 2 = 1 past it
    assert ev.peaks(_t({2: 0.5, 3: 2.0, 4: 1.0, 5: 0.5, 6: 0.1}), _t({})) == [3]
    # below the short threshold (1.4): never valid, never emitted
    assert ev.peaks(_t({2: 0.5, 3: 1.3, 4: 0.5}), _t({})) == []
    # a rise of exactly the peak height opens no candidate
    assert ev.peaks(_t({3: 0.2, 4: 5.0, 5: 0.0}), _t({})) == [4]
    assert ev.peaks(_t({3: 0.2}), _t({})) == []
    # long detector alone: valid at 9, emitted at 12 (more than 6 // 2 past 8)
    assert ev.peaks(_t({}), _t({8: 10.0, 9: 5.0, 10: 1.0})) == [8]
    assert ev.peaks(_t({}, 13), _t({8: 10.0, 9: 5.0, 10: 1.0}, 13)) == [8]
    assert ev.peaks(_t({}, 12), _t({8: 10.0, 9: 5.0, 10: 1.0}, 12)) == []
    # the long detector's threshold is 9.0
    assert ev.peaks(_t({}), _t({8: 8.9, 9: 1.0})) == []
    # a short peak above 1.4 masks the long detector up to its position + 6
    # and resets it: the long peak at 5 is never seen; after the mask the long
    # detector needs a rise from a minimum again (at 10 a peak is taken as
    # the first minimum, at 11 it rises from the 0 at 10)
    assert ev.peaks(_t({2: 0.5, 3: 2.0, 4: 0.5}), _t({5: 12.0, 6: 1.0})) == [3]
    assert ev.peaks(_t({2: 0.5, 3: 2.0, 4: 0.5}), _t({10: 12.0, 11: 1.0})) == [3]
    assert ev.peaks(_t({2: 0.5, 3: 2.0, 4: 0.5}), _t({11: 12.0, 12: 1.0})) == [3, 11]
    # both detectors on the same position: one boundary
    assert ev.peaks(_t({2: 0.5, 3: 20.0, 4: 0.5}, 12), _t({3: 20.0, 4: 1.0}, 12)) == [3]


@pytest.mark.parametrize("minlen", [3, 5, 9])
def test_noise_free_steps_recovered_exactly(minlen):
    rng = np.random.default_rng(minlen)
    for _ in range(10):
        lens = rng.integers(minlen, 16, size=40)
        lv = rng.normal(90, 12, size=40).astype(np.float32)
        x = np.repeat(lv, lens)
        assert ev.boundaries(x) == list(np.cumsum(lens)[:-1])
        e = ev.events(x)
        assert np.array_equal(e, lv)
        assert np.array_equal(ev.query_events(x, trim=5, keep=20), lv[5:25])


def test_partition_and_means_on_noisy_reads():
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(g, synth.make_level_table(), 6, 120, 0.5, 3)
    for r in range(raw.nreads):
        x = raw.values[raw.offsets[r]:raw.offsets[r + 1]]
        b = ev.boundaries(x)
        assert b == sorted(set(b)) and all(0 < v < x.size for v in b)
        e = ev.events(x)
        assert e.size == len(b) + 1
        cuts = [0] + b + [x.size]
        want = [np.mean(x[a:c].astype(np.float64)) for a, c in zip(cuts[:-1], cuts[1:])]
        assert np.allclose(e, want, rtol=1e-6)
        # the short detector splits levels (noise in 3-sample windows) more
        # often than it merges similar neighbours: 1-2.5 events per level
        assert raw.levels[r].size < e.size < 2.5 * raw.levels[r].size


def test_short_and_empty_reads():
    assert ev.boundaries(np.zeros(0, np.float32)) == []
    assert ev.events(np.zeros(0, np.float32)).size == 0
    assert ev.events(np.array([4.0], np.float32)).tolist() == [4.0]
    assert ev.query_events(np.arange(5, dtype=np.float32), trim=1, keep=3).size == 0


def test_detected_events_align_where_the_read_came_from():
    g = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    table = synth.make_level_table()
    raw = synth.simulate_raw(g, table, 8, 320, 1.0, 5)
    _, ref, _ = oracle.prepare_reference(g, table, synth.K)
    nk = synth.SMALL_GENOME - synth.K + 1
    inside = 0
    for r in range(raw.nreads):
        x = raw.values[raw.offsets[r]:raw.offsets[r + 1]]
        e = ev.query_events(x, trim=50, keep=250)
        assert e.size == 250
        q, _ = oracle.quantize(oracle.znorm(e), 64.0)
        _, end = oracle.sdtw_i64(q, ref)
        # the 250 events after the adaptor lie within the read's 320 bases
        first = int(raw.strand[r]) * nk + int(raw.start[r])
        inside += first + 60 <= end <= first + 320
    assert inside >= 7, inside
