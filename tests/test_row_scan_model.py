"""CPU model of the whole-device single-query scheme (sdtw_align_one_wide),
checked against the oracle: each row as a scan of maps x -> min(a, x + d)
over column tiles, per-thread strips, a two-level look-back (tiles within a
group, then group maps) over flags that appear in random orders, and the
saturated sums of the look-back.  Small tiles, groups and windows stand in
for the kernel's 256 x C columns, 64-tile groups and 64-lane windows, so
that every path is taken on small inputs.  No GPU.
"""
import numpy as np
import pytest

import oracle

INF = 1 << 31
IDN = (INF, 0)


def comp(f, g, cap=None):
    """f, then g; with cap, the summed distances saturate there."""
    d = f[1] + g[1]
    return (min(g[0], f[0] + g[1]), d if cap is None else min(d, cap))


def flag_roundtrip(f, dbits):
    """A map published in a flag word and read back: status in the low two
    bits, d in the next dbits bits, a above them (the kernel's 64-bit word
    has dbits = 30 and a in the high 32 bits).  A d that does not fit in its
    field spills into a's lowest bit and reads back truncated."""
    w = (f[0] << (dbits + 2)) | (f[1] << 2) | 1
    return (w >> (dbits + 2), (w & ((1 << (dbits + 2)) - 1)) >> 2)


def look_back(t, agg, inc, gag, GT, GW, rng, cap, dbits):
    """x entering tile t, or None while a flag it needs is missing."""
    def seen(p):  # an inc flag may be published but not yet visible
        return p in inc and (p == 0 or rng.random() < 0.6)
    if t == 0:
        return INF
    first = t - t % GT
    closer = t - first == GT - 1
    acc = IDN
    if t > first:
        lanes = [t - 1 - k for k in range(GT) if t - 1 - k >= first]
        kn = next((k for k, p in enumerate(lanes) if seen(p)), None)
        k = len(lanes) if (closer or kn is None) else kn
        if any(lanes[j] not in agg for j in range(k)):
            return None
        win = IDN
        for j in reversed(range(k)):
            win = comp(win, agg[lanes[j]], cap)
        if closer:
            gag[t // GT] = flag_roundtrip(comp(win, agg[t], cap), dbits)
        if kn is not None:
            part = IDN
            for j in reversed(range(kn)):
                part = comp(part, agg[lanes[j]], cap)
            return min(part[0], inc[lanes[kn]] + part[1])
        acc = win
    elif closer:
        gag[t // GT] = agg[t]  # already a published word
    gbase, gacc = t // GT - 1, IDN
    while True:
        lanes = [gbase - k for k in range(GW)]
        k, edge = None, False
        for j, g in enumerate(lanes):
            if g < 0:
                k, edge = j, True
                break
            if seen(g * GT + GT - 1):
                k = j
                break
        kk = GW if k is None else k
        if any(lanes[j] not in gag for j in range(kk)):
            return None
        win = IDN
        for j in reversed(range(kk)):
            win = comp(win, gag[lanes[j]], cap)
        gacc = comp(win, gacc, cap)
        if k is not None:
            v = INF if edge else inc[lanes[k] * GT + GT - 1]
            xg = min(gacc[0], v + gacc[1])
            return min(acc[0], xg + acc[1])
        gbase -= GW


def row_scan_sdtw(q, ref, C, TH, GT, GW, seed, cap=(1 << 30) - 1, dbits=30, row=None,
                  return_row=False, left_of_tile=None):
    """(cost, end) of q against ref; with ``row`` (a resident row, the last
    row of the rows before q) the rows of q extend it.  ``return_row``: the
    new last row as well, (cost, end, row)."""
    rng = np.random.default_rng(seed)
    x_all = q.astype(np.int64) + 32768
    y = ref.astype(np.int64) + 32768
    n, T = y.size, C * TH
    ntiles = (n + T - 1) // T
    ycols = np.zeros(ntiles * T, np.int64)
    ycols[:n] = y
    prev = np.zeros((ntiles, T), np.int64)   # gamma(0, j) = 0
    xprev = np.zeros(ntiles, np.int64)        # gamma(i-1, first column - 1)
    if row is not None:
        # the old row, and the old value left of each tile (+inf left of
        # column 0), as the clearing kernel takes it aside
        prev.reshape(-1)[:n] = row
        xprev[0] = INF
        xprev[1:] = [row[t * T - 1] for t in range(1, ntiles)]
        if left_of_tile is not None:  # (a planted mistake's values)
            xprev[1:] = left_of_tile[1:]
    for x in x_all:
        d = np.abs(int(x) - ycols.reshape(ntiles, T))
        left = np.concatenate([xprev[:, None], prev[:, :-1]], axis=1)
        a = d + np.minimum(left, prev)
        agg, inc, gag, before = {}, {}, {}, {}
        for t in range(ntiles):
            maps = []
            for th in range(TH):
                m = IDN
                for c in range(th * C, th * C + C):
                    m = comp(m, (int(a[t, c]), int(d[t, c])))
                maps.append(m)
            acc, ex = IDN, []
            for m in maps:
                ex.append(acc)
                acc = comp(acc, m)
            agg[t], before[t] = flag_roundtrip(acc, dbits), ex
        xin, pending = {}, list(rng.permutation(ntiles))
        while pending:
            t = int(pending.pop(0))
            v = look_back(t, agg, inc, gag, GT, GW, rng, cap, dbits)
            if v is None:
                pending.append(t)
                continue
            xin[t] = v
            inc[t] = min(agg[t][0], v + agg[t][1])
        for t in range(ntiles):
            for th in range(TH):
                carry = min(before[t][th][0], xin[t] + before[t][th][1])
                for c in range(th * C, th * C + C):
                    carry = min(int(a[t, c]), carry + int(d[t, c]))
                    prev[t, c] = carry
            xprev[t] = xin[t]
    last = prev.reshape(-1)[:n]
    j = int(np.argmin(last))
    if return_row:
        return int(last[j]), j, last.copy()
    return int(last[j]), j


@pytest.mark.parametrize("case", range(40))
def test_model_matches_oracle(case):
    rng = np.random.default_rng(case)
    n, m = int(rng.integers(1, 260)), int(rng.integers(1, 7))
    C, TH = int(rng.choice([1, 2, 3])), int(rng.choice([1, 2, 4]))
    GT, GW = int(rng.choice([1, 2, 3, 4])), int(rng.choice([1, 2, 3]))
    lo = int(rng.choice([2, 30, 32768]))
    ref = rng.integers(-lo, lo, size=n).astype(np.int16)
    q = rng.integers(-lo, lo, size=m).astype(np.int16)
    assert row_scan_sdtw(q, ref, C, TH, GT, GW, case) == oracle.sdtw_i64(q, ref)


@pytest.mark.parametrize("case", range(12))
def test_model_extends_a_resident_row(case):
    # chunk by chunk from the resident row: cost, end and the row after each
    # chunk equal the oracle's on the concatenated prefix
    rng = np.random.default_rng(500 + case)
    n = int(rng.integers(1, 200))
    C, TH = int(rng.choice([1, 2, 3])), int(rng.choice([1, 2, 4]))
    GT, GW = int(rng.choice([1, 2, 4])), int(rng.choice([1, 2]))
    ref = rng.integers(-300, 300, size=n).astype(np.int16)
    chunks = [rng.integers(-300, 300, size=int(m)).astype(np.int16)
              for m in rng.integers(1, 5, size=3)]
    row = None  # the first chunk starts from the free-start zeros
    for k, ck in enumerate(chunks):
        c, e, row = row_scan_sdtw(ck, ref, C, TH, GT, GW, case + k, row=row, return_row=True)
        pre = np.concatenate(chunks[:k + 1])
        want_c, want_e, want_row = oracle.sdtw_i64(pre, ref, lastrow=True)
        assert (c, e) == (want_c, want_e)
        assert np.array_equal(row, want_row)


def test_resident_row_diagonal_left_of_a_tile_matters():
    # the first new row's diagonal at a tile's first column is the old row's
    # value left of the tile; taking the new value there instead (as a tile
    # that starts after its left neighbour wrote back would) changes results
    rng = np.random.default_rng(7)
    bad = 0
    for s in range(20):
        ref = rng.integers(-300, 300, size=48).astype(np.int16)
        a = rng.integers(-300, 300, size=3).astype(np.int16)
        b = rng.integers(-300, 300, size=3).astype(np.int16)
        _, _, row_a = oracle.sdtw_i64(a, ref, lastrow=True)
        _, _, row_ab = oracle.sdtw_i64(np.concatenate([a, b]), ref, lastrow=True)
        _, _, row = row_scan_sdtw(b, ref, 2, 2, 2, 2, s, row=row_a, return_row=True)
        assert np.array_equal(row, row_ab)
        # the planted mistake: each tile's left value (tiles of 4 columns)
        # read from the row as its left neighbour wrote it back
        _, _, row_new = oracle.sdtw_i64(np.concatenate([a, b[:1]]), ref, lastrow=True)
        lefts = [0] + [int(row_new[t * 4 - 1]) for t in range(1, 12)]
        _, _, row2 = row_scan_sdtw(b[:1], ref, 2, 2, 2, 2, s, row=row_a, return_row=True,
                                   left_of_tile=np.array(lefts))
        bad += not np.array_equal(row2, row_new)
    assert bad > 0


def test_saturated_sums_do_not_change_results():
    # a cap far below the summed distances, still above every cost
    rng = np.random.default_rng(99)
    ref = rng.integers(-30, 30, size=200).astype(np.int16)
    q = rng.integers(-30, 30, size=5).astype(np.int16)
    want = oracle.sdtw_i64(q, ref)
    assert row_scan_sdtw(q, ref, 2, 2, 2, 2, 5, cap=1024) == want


def test_planted_mistake_is_caught():
    # composing a window nearest-first instead of farthest-first is wrong
    global comp
    ok = comp
    try:
        comp = lambda f, g, cap=None: ok(g, f, cap)  # noqa: E731
        rng = np.random.default_rng(4)
        bad = 0
        for s in range(10):
            ref = rng.integers(-30, 30, size=60).astype(np.int16)
            q = rng.integers(-30, 30, size=4).astype(np.int16)
            bad += row_scan_sdtw(q, ref, 2, 2, 2, 2, s) != oracle.sdtw_i64(q, ref)
        assert bad > 0
    finally:
        comp = ok


def test_group_maps_saturate_within_their_flag_field():
    # Group maps saturate D at the largest value their flag field holds.  The
    # field is narrowed here (15 bits) so that small groups reach the cap.
    # Query (0, 500, 1000); the reference is one group of (0, 500) pairs, two
    # groups of -1000 (their summed distances exceed the field) and one group
    # of (500, 1000) pairs: the best cost is 500.  A path that skipped the
    # middle groups for free would reach 0, which is what a map whose D spilt
    # out of its field (a cap of 2^bits instead of 2^bits - 1) hands the
    # tiles to the right whenever they look back over a saturated group.
    bits, TH, C, GT = 15, 4, 3, 4
    group = TH * C * GT
    ref = np.array([0, 500] * (group // 2) + [-1000] * (2 * group) +
                   [500, 1000] * (group // 2), np.int16)
    q = np.array([0, 500, 1000], np.int16)
    want = oracle.sdtw_i64(q, ref)
    assert want == (500, 1)
    fails = 0
    for s in range(10):
        assert row_scan_sdtw(q, ref, C, TH, GT, 2, s, cap=(1 << bits) - 1, dbits=bits) == want
        fails += row_scan_sdtw(q, ref, C, TH, GT, 2, s, cap=1 << bits, dbits=bits) != want
    assert fails > 0
    # random values with the narrowed field and the right cap
    rng = np.random.default_rng(100)
    for s in range(6):
        ref = rng.integers(-1000, 1000, size=480).astype(np.int16)
        q = rng.integers(-1000, 1000, size=3).astype(np.int16)
        assert row_scan_sdtw(q, ref, C, TH, GT, 2, s, cap=(1 << bits) - 1,
                             dbits=bits) == oracle.sdtw_i64(q, ref)
