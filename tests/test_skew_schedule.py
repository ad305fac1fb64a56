"""CPU model of the continuous-skew lane schedule of the alignment kernel.

The model replays, lane by lane in NumPy, what the batch kernel's 64 lanes do
for K chains per lane (lane l's strip of W columns is cut into K sub-strips
of W/K columns; sub-strip h of lane l is "sub-lane" s = K l + h and works on
row t - s at step t, so a lane advances K independent dependency chains per
step).  It follows the kernel's periods of M steps: the 64K switch steps in
which sub-lane r enters its next tile -- either every switch at the top of
its own step (the one-band kernel), or sub-lane 0 there and every later
sub-lane's switch issued during the step before, once it has computed its
last row on the old tile, except the previous-row reload of its last group
of columns, done after its outgoing edge has been read by its right
neighbour (the kernel with bands or a resident row) -- the query/boundary
LDS entries at K(63 - l) + r + (K - 1 - h) read one step ahead, the boundary
writes of the last sub-lane (at r, or r + M while its row wraps), the
reference values of the next tile held apart from the staged last rows
(switch groups of 8 columns, as the kernel's), the
per-tile fold of the staged last rows and the lexicographic final
reduction.  At a tile switch the previous row gamma(0, .) = 0 is entered as
the kernel does it: every other column cleared and the diagonal set to 0,
so that every cell of the tile's first row has a zero among its minimum's
operands.  It checks the schedule itself against the oracle on the CPU; the
GPU parity tests check the compiled kernel.
"""
import numpy as np
import pytest

import oracle

INF = 0xFFFFFFFF


def skew_model(x, yref, W, K=1, defer_last=True, pipe=True, gc=8, clear_diag=True):
    L = 64
    T = L * W
    H = W // K
    S = L * K  # sub-lanes
    M, N = len(x), len(yref)
    assert M >= S + 1 and W % K == 0
    ntiles = (N + T - 1) // T
    ref = np.zeros(ntiles * T + T, np.uint64)
    ref[:N] = yref.astype(np.int64) + 32768
    xb = x.astype(np.int64) + 32768
    nent = M + S
    bxx = np.array([xb[(k - (S - 1)) % M] for k in range(nent)], np.uint64)
    bxy = np.full(nent, INF, np.uint64)
    stage = np.zeros((L, W), np.uint64)       # finished last rows of the tile
    ynext = ref[0:T].reshape(L, W).copy()     # reference values of the next tile
    y = np.zeros((L, W), np.uint64)
    G = min(gc, H)                            # columns of the deferred last group
    a = np.zeros((L, W), np.uint64)
    b = np.zeros((L, W), np.uint64)
    dprev = np.full((K, L), INF, np.uint64)
    best = np.full(L, INF, np.uint64)
    bestj = np.full(L, 2 ** 31 - 1, np.int64)
    lanes = np.arange(L)
    base = K * (63 - lanes)

    def entries(r):
        ks = [base + r + (K - 1 - h) for h in range(K)]
        return [(bxx[k].copy(), bxy[k].copy()) for k in ks]

    st = {"next": None}

    def clear(row, l, c0, c1):
        # gamma(0, .) = 0 entered as the kernel does: the odd columns cleared
        row[l, [c for c in range(c0, c1) if c % 2 == 1]] = 0

    def enter(l, h, row, c1):
        # sub-lane (l, h) enters its next tile: the finished row out, the new
        # reference values in, the previous row of columns [h H, c1) cleared
        cols = slice(h * H, (h + 1) * H)
        stage[l, cols] = row[l, cols]
        y[l, cols] = ynext[l, cols]
        clear(row, l, h * H, c1)

    def step(r, up, nw, write_b, wrap, sw):
        ent = st["next"]  # read one step earlier
        st["next"] = entries(r + 1)
        lefts = []
        for h in range(K):
            lf = np.empty(L, np.uint64)
            if h == 0:  # lane l-1's last sub-strip edge; lane 0: boundary column
                lf[1:] = up[:-1, W - 1]
                lf[0] = ent[0][1][0]
            else:       # own previous sub-strip edge, computed one step earlier
                lf[:] = up[:, h * H - 1]
            lefts.append(lf)
        if sw and r < S:  # sub-lane r enters its next tile
            l, h = r // K, r % K
            if r == 0 or not pipe:  # all of the switch, here
                enter(l, h, up, (h + 1) * H)
                if clear_diag:
                    dprev[h][l] = 0
            elif defer_last:
                # issued during the previous step, but for the last group's
                # previous row, cleared now that the right neighbours have
                # read their edge from it
                clear(up, l, (h + 1) * H - G, (h + 1) * H)
        for h in range(K):
            ex = ent[h][0]
            diag, lf = dprev[h].copy(), lefts[h].copy()
            for w in range(h * H, (h + 1) * H):
                m = np.minimum(np.minimum(up[:, w], diag), lf)
                d = np.abs(ex.astype(np.int64) - y[:, w].astype(np.int64)).astype(np.uint64)
                c = (d + m) & 0xFFFFFFFF
                nw[:, w] = c
                diag, lf = up[:, w], c
            dprev[h] = lefts[h]
        if write_b:
            bxy[r + (M if wrap else 0)] = nw[63, W - 1]
        if sw and pipe and r + 1 < S:
            # sub-lane r + 1 has computed its last row on the old tile; its
            # switch is issued in this step, but for the last group's previous
            # row (its right neighbours still read their edge there)
            l, h = (r + 1) // K, (r + 1) % K
            enter(l, h, nw, (h + 1) * H - (G if defer_last else 0))
            if clear_diag:
                dprev[h][l] = 0

    p = 0
    while True:
        st["next"] = entries(0)  # fresh read at the start of every period
        for r in range(0, S, 2):
            step(r, a, b, p > 0 or r == S - 1, r != S - 1, True)
            step(r + 1, b, a, p > 0 or r + 1 == S - 1, r + 1 != S - 1, True)
        if p >= 1:
            for l in range(L):
                for w in range(W):
                    j = (p - 1) * T + l * W + w
                    if j < N and stage[l, w] < best[l]:
                        best[l], bestj[l] = stage[l, w], j
        if p + 1 < ntiles:  # every lane has entered tile p: fetch tile p + 1
            ynext[:] = ref[(p + 1) * T:(p + 2) * T].reshape(L, W)
        if p == ntiles:
            break
        r = S
        while r + 1 < M:
            step(r, a, b, True, False, False)
            step(r + 1, b, a, True, False, False)
            r += 2
        if r < M:
            step(r, a, b, True, False, False)
            a[:] = b
        p += 1
    i = np.lexsort((bestj, best))[0]
    return int(best[i]), int(bestj[i])


@pytest.mark.parametrize("W,K,M,N,lo,hi", [
    (4, 1, 65, 1, -2, 2), (4, 1, 65, 257, -2, 2), (4, 1, 65, 255, -30000, 30000),
    (8, 1, 66, 513, -50, 50), (4, 1, 131, 700, -3, 3), (8, 1, 97, 1100, -30000, 30000),
    (16, 1, 70, 1025, -5, 5),
    (4, 2, 129, 1, -2, 2), (4, 2, 129, 300, -3, 3), (8, 2, 130, 1100, -30000, 30000),
    (16, 2, 200, 2049, -5, 5), (8, 2, 257, 600, -40, 40), (8, 4, 257, 900, -3, 3),
])
@pytest.mark.parametrize("pipe", [True, False])
def test_skew_schedule_matches_oracle(W, K, M, N, lo, hi, pipe):
    rng = np.random.default_rng(W * 1000 + K * 100 + M + N)
    x = rng.integers(lo, hi, size=M).astype(np.int16)
    y = rng.integers(lo, hi, size=N).astype(np.int16)
    assert skew_model(x, y, W, K, pipe=pipe) == oracle.sdtw_i64(x, y)


@pytest.mark.parametrize("gc", [4, 16])
def test_other_switch_group_sizes(gc):
    # the kernel issues a switch in groups of 8 columns; the schedule holds
    # for other group sizes too
    rng = np.random.default_rng(gc)
    for W, K, M, N in ((16, 1, 70, 1025), (8, 1, 66, 513), (16, 2, 200, 900), (32, 1, 70, 2100)):
        x = rng.integers(-40, 40, size=M).astype(np.int16)
        y = rng.integers(-40, 40, size=N).astype(np.int16)
        assert skew_model(x, y, W, K, gc=gc) == oracle.sdtw_i64(x, y)


@pytest.mark.parametrize("K", [1, 2, 4])
def test_prefetch_needs_one_more_row_than_sublanes(K):
    # During step r lane 0 prefetches the boundary row r + 1 of its period
    # while the last sub-lane (S - 1) writes row (r - (S - 1)) mod M.  They
    # collide (a stale read) exactly when M = S, which is why the kernel takes
    # M >= S + 1; with M >= S + 1 the row was written at least two steps
    # before it is read.
    S = 64 * K
    for M in (S, S + 1, S + 7, 3 * S):
        collide = any((r + 1) % M == (r - (S - 1)) % M for r in range(M))
        assert collide == (M == S)


def test_clearing_without_the_diagonal_is_caught():
    # a planted schedule mistake: every other column cleared but the
    # diagonal left as it was, so a strip's first cell can miss its zero
    rng = np.random.default_rng(78)
    bad = 0
    for _ in range(4):
        x = rng.integers(-30, 30, size=70).astype(np.int16)
        y = rng.integers(-30, 30, size=600).astype(np.int16)
        want = oracle.sdtw_i64(x, y)
        assert skew_model(x, y, 4, 1) == want
        bad += skew_model(x, y, 4, 1, clear_diag=False) != want
    assert bad > 0


def test_reloading_the_edge_columns_early_is_caught():
    # a planted schedule mistake: the whole previous row reloaded during the
    # step before the switch, so the right neighbour reads a zero as its
    # edge instead of the finished row's last value
    rng = np.random.default_rng(77)
    bad = 0
    for _ in range(4):
        x = rng.integers(-30, 30, size=70).astype(np.int16)
        y = rng.integers(-30, 30, size=600).astype(np.int16)
        want = oracle.sdtw_i64(x, y)
        assert skew_model(x, y, 4, 1) == want
        bad += skew_model(x, y, 4, 1, defer_last=False) != want
    assert bad > 0
