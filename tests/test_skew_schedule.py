"""CPU model of the continuous-skew lane schedule of the alignment kernel.

The model replays, lane by lane in NumPy, what the batch kernel's 64 lanes do
for K chains per lane (lane l's strip of W columns is cut into K sub-strips
of W/K columns; sub-strip h of lane l is "sub-lane" s = K l + h and works on
row t - s at step t, so a lane advances K independent dependency chains per
step).  It follows the kernel's periods of M steps: the 64K switch steps in
which sub-lane r enters its next tile (after its outgoing edge has been read
by its right neighbour), the query/boundary LDS entries at K(63 - l) + r +
(K - 1 - h) read one step ahead, the boundary writes of the last sub-lane (at
r, or r + M while its row wraps), the per-tile fold of the staged last rows
and the lexicographic final reduction.  At a tile switch the previous row is
cleared the way the kernel clears it (the diagonal and every other column
only), so the model also checks that a zero among each cell's minimum
operands is all the first row of a tile needs.  It checks the schedule
itself against the oracle on the CPU; the GPU parity tests check the
compiled kernel.
"""
import numpy as np
import pytest

import oracle

INF = 0xFFFFFFFF


def skew_model(x, yref, W, K=1):
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
    stage = ref[0:T].reshape(L, W).copy()
    y = np.zeros((L, W), np.uint64)
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
            cols = slice(h * H, (h + 1) * H)
            nv = stage[l, cols].copy()
            stage[l, cols] = up[l, cols]
            y[l, cols] = nv
            # the previous row of a tile is gamma(0, .) = 0; like the kernel,
            # clear only the diagonal and every other column (offsets 1, 3,
            # ...) and leave the finished row's values in the others: each
            # cell's minimum still has a zero operand
            up[l, h * H + 1:(h + 1) * H:2] = 0
            dprev[h][l] = 0
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
        if p + 1 < ntiles:
            stage[:] = ref[(p + 1) * T:(p + 2) * T].reshape(L, W)
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
def test_skew_schedule_matches_oracle(W, K, M, N, lo, hi):
    rng = np.random.default_rng(W * 1000 + K * 100 + M + N)
    x = rng.integers(lo, hi, size=M).astype(np.int16)
    y = rng.integers(lo, hi, size=N).astype(np.int16)
    assert skew_model(x, y, W, K) == oracle.sdtw_i64(x, y)


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
