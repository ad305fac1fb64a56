"""One query over the whole device (sdtw_align_one_wide): row scans with a
look-back between column tiles.  Bit-exact against the exact integer oracle
(cost and end) for every tile width, across tile edges and ragged tails, with
ties, with the extreme int16 values that make a tile's summed distances
largest, and on references long enough that the look-back saturates its
summed distances.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")

COLS = [8, 16, 32, 64]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.load_library()
    return torch.device("cuda:0")


def run_wide(dev, ref_np, q_np, cols):
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    try:
        c, e = sd.align_one_wide(ref, torch.from_numpy(q_np).to(dev), cols=cols)
        torch.cuda.synchronize()
        return int(c.item()), int(e.item())
    finally:
        ref.close()


@pytest.mark.parametrize("cols", COLS + [0])
@pytest.mark.parametrize("n,m", [(1, 1), (1, 7), (5, 1), (2047, 63), (2048, 64), (2049, 65),
                                 (16383, 250), (16385, 3), (40001, 130)])
def test_random_sizes(dev, n, m, cols):
    rng = np.random.default_rng(n * 31 + m + cols)
    ref = rng.integers(-3000, 3000, size=n).astype(np.int16)
    q = rng.integers(-3000, 3000, size=m).astype(np.int16)
    note(f"wide n={n} m={m} cols={cols}")
    assert run_wide(dev, ref, q, cols) == oracle.sdtw_i64(q, ref)


@pytest.mark.parametrize("cols", COLS)
def test_on_target_read_small_genome(dev, cols):
    w = synth.workload(0)
    _, ref, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    _, q, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    note(f"wide on-target read vs {ref.size} columns, cols={cols}")
    got = run_wide(dev, ref, q, cols)
    assert got == oracle.sdtw_i64(q, ref)
    assert abs(got[1] - int(w.reads.end_true[0])) <= 10


@pytest.mark.parametrize("cols", [8, 64])
def test_ties_first_end_wins(dev, cols):
    # a three-letter alphabet: many columns share the minimum
    rng = np.random.default_rng(3)
    ref = rng.integers(0, 3, size=70001).astype(np.int16)
    for m in (1, 2, 5, 64, 300):
        q = rng.integers(0, 3, size=m).astype(np.int16)
        note(f"wide ties m={m} cols={cols}")
        assert run_wide(dev, ref, q, cols) == oracle.sdtw_i64(q, ref)
    ref = np.zeros(40000, np.int16)  # every column ties
    assert run_wide(dev, ref, np.zeros(9, np.int16), cols) == (0, 0)


@pytest.mark.parametrize("cols", [16, 64])
def test_extremes_longest_query(dev, cols):
    # |x - y| = 65,535 everywhere a value flips: the largest costs (M = 4,096)
    # and the largest per-tile sums of distances
    rng = np.random.default_rng(11)
    ref = np.where(rng.random(50000) < 0.5, 32767, -32768).astype(np.int16)
    q = np.where(rng.random(4096) < 0.5, -32768, 32767).astype(np.int16)
    note(f"wide extremes M=4096 N=50000 cols={cols}")
    assert run_wide(dev, ref, q, cols) == oracle.sdtw_i64(q, ref)


def test_saturated_lookback_long_reference(dev):
    # 3 M columns of alternating extremes: tiles to the right of the best end
    # see summed distances far above 2^30 in their look-back
    n = 3_000_000
    ref = np.full(n, 32767, np.int16)
    ref[::2] = -32768
    ref[1_234_567] = 0
    q = np.array([0, 0, 5, -5, 32767, -32768, 0, 0], np.int16)
    for cols in (8, 64):
        note(f"wide saturated look-back N={n} cols={cols}")
        assert run_wide(dev, ref, q, cols) == oracle.sdtw_i64(q, ref)


def test_low_register_form_on_long_reference(dev):
    # more 32-column tiles than the plain form keeps resident (4.2 M columns
    # on MI355X): the launch takes the low-register form of the kernel
    rng = np.random.default_rng(31)
    n = 5_000_000
    ref = rng.integers(-2000, 2000, size=n).astype(np.int16)
    q = rng.integers(-2000, 2000, size=12).astype(np.int16)
    ref[4_400_000:4_400_012] = q  # an exact occurrence near the end
    want = oracle.sdtw_i64(q, ref)
    assert want == (0, 4_400_011)
    for cols in (32, 0):
        note(f"wide low-register form N={n} cols={cols}")
        assert run_wide(dev, ref, q, cols) == want


def test_back_to_back_calls_share_scratch(dev):
    # the scratch of a finished call is reused: a large call, then smaller
    # ones on another reference, then the large one again
    rng = np.random.default_rng(21)
    big = rng.integers(-500, 500, size=300_000).astype(np.int16)
    small = rng.integers(-500, 500, size=3000).astype(np.int16)
    qb = rng.integers(-500, 500, size=400).astype(np.int16)
    qs = rng.integers(-500, 500, size=20).astype(np.int16)
    rb = sd.Reference(torch.from_numpy(big).to(dev))
    rs = sd.Reference(torch.from_numpy(small).to(dev))
    outs = []
    for r, q, cols in ((rb, qb, 8), (rs, qs, 64), (rs, qb, 16), (rb, qs, 0), (rb, qb, 32)):
        c, e = sd.align_one_wide(r, torch.from_numpy(q).to(dev), cols=cols)
        outs.append((c, e))
    torch.cuda.synchronize()
    want = [oracle.sdtw_i64(qb, big), oracle.sdtw_i64(qs, small), oracle.sdtw_i64(qb, small),
            oracle.sdtw_i64(qs, big), oracle.sdtw_i64(qb, big)]
    assert [(int(c.item()), int(e.item())) for c, e in outs] == want
    rb.close()
    rs.close()


def test_matches_single_wave_kernel(dev):
    w = synth.workload(1, nq=6)
    _, ref, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    _, q, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    r = sd.Reference(torch.from_numpy(ref).to(dev))
    for i in range(6):
        qi = torch.from_numpy(q[w.reads.offsets[i]:w.reads.offsets[i + 1]]).to(dev)
        a = [int(t.item()) for t in sd.align_one(r, qi)]
        b = [int(t.item()) for t in sd.align_one_wide(r, qi)]
        assert a == b
    r.close()


def test_float_reference_rejected(dev):
    r = sd.Reference(torch.zeros(100, dtype=torch.float32, device=dev))
    with pytest.raises(sd.SdtwError):
        sd.align_one_wide(r, torch.zeros(5, dtype=torch.int16, device=dev))
    r.close()


@pytest.mark.parametrize("cols", [8, 16])
def test_free_skip_over_saturated_groups_is_impossible(dev, cols):
    # Query (0, 500, 1000).  Reference: one look-back group (64 tiles) of
    # (0, 500) pairs, two groups of -30000 (each group's summed distances far
    # above 2^30, so its map saturates), one group of (500, 1000) pairs.  The
    # best cost is 500 (end at column 1).  A group map whose saturated sum
    # read back as 0 would let the right-hand tiles start from the left
    # group's cost 0 and report 0.
    group = 64 * 256 * cols
    ref = np.concatenate([np.tile(np.array([0, 500], np.int16), group // 2),
                          np.full(2 * group, -30000, np.int16),
                          np.tile(np.array([500, 1000], np.int16), group // 2)])
    q = np.array([0, 500, 1000], np.int16)
    want = oracle.sdtw_i64(q, ref)
    assert want == (500, 1)
    note(f"wide saturated groups N={ref.size} cols={cols}")
    for _ in range(3):
        assert run_wide(dev, ref, q, cols) == want


def test_random_extremes_over_many_groups(dev):
    # random extreme codes over 2.3 groups of 8-column tiles: every group map
    # saturates
    rng = np.random.default_rng(41)
    ref = np.where(rng.random(300_000) < 0.5, 32767, -32768).astype(np.int16)
    ref[rng.integers(0, ref.size, size=3000)] = 0
    q = rng.integers(-32768, 32767, size=40).astype(np.int16)
    note("wide random extremes N=300000 cols=8")
    assert run_wide(dev, ref, q, 8) == oracle.sdtw_i64(q, ref)
