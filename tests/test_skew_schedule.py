"""CPU model of the continuous-skew lane schedule of the alignment kernel.

The model replays, lane by lane in NumPy, what the batch kernel's 64 lanes do:
periods of M steps, the 64 switch steps in which lane r enters its next tile
(its last-row edge read by lane r+1 before the switch), the query/boundary LDS
entries at 63 + r - l, lane 63's boundary writes (at r, or r + M while its
row wraps), the per-tile fold of the staged last rows and the lexicographic
final reduction.  It checks the schedule itself against the oracle on the
CPU; the GPU parity tests check the compiled kernel.
"""
import numpy as np
import pytest

import oracle

INF = 0xFFFFFFFF


def skew_model(x, yref, W):
    L = 64
    T = L * W
    M, N = len(x), len(yref)
    assert M >= 65
    ntiles = (N + T - 1) // T
    ref = np.zeros(ntiles * T + T, np.uint64)
    ref[:N] = yref.astype(np.int64) + 32768
    xb = x.astype(np.int64) + 32768
    bxx = np.array([xb[(k - 63) % M] for k in range(M + 65)], np.uint64)
    bxy = np.full(M + 65, INF, np.uint64)
    stage = ref[0:T].reshape(L, W).copy()
    y = np.zeros((L, W), np.uint64)
    a = np.zeros((L, W), np.uint64)
    b = np.zeros((L, W), np.uint64)
    st = {"dprev": np.full(L, INF, np.uint64), "next": None}
    best = np.full(L, INF, np.uint64)
    bestj = np.full(L, 2 ** 31 - 1, np.int64)
    lanes = np.arange(L)

    def step(r, up, nw, write_b, wrap, sw):
        # this step's entries were read one step earlier (prefetch), before
        # the previous step's boundary write became visible to this read
        ex, ey = st["next"]
        k = 63 + r + 1 - lanes
        st["next"] = (bxx[k].copy(), bxy[k].copy())
        left = np.empty(L, np.uint64)
        left[1:] = up[:-1, W - 1]
        left[0] = ey[0]
        if sw and r < 64:  # lane r enters its next tile
            nv = stage[r].copy()
            stage[r] = up[r]
            y[r] = nv
            up[r] = 0
        diag, lf = st["dprev"].copy(), left.copy()
        for w in range(W):
            m = np.minimum(np.minimum(up[:, w], diag), lf)
            d = np.abs(ex.astype(np.int64) - y[:, w].astype(np.int64)).astype(np.uint64)
            c = (d + m) & 0xFFFFFFFF
            nw[:, w] = c
            diag, lf = up[:, w], c
        st["dprev"] = left
        if write_b:
            bxy[r + (M if wrap else 0)] = nw[63, W - 1]

    p = 0
    while True:
        k0 = 63 - lanes  # fresh read at the start of every period
        st["next"] = (bxx[k0].copy(), bxy[k0].copy())
        for r in range(0, 64, 2):
            step(r, a, b, p > 0, True, True)
            step(r + 1, b, a, p > 0 or r + 1 == 63, r + 1 != 63, True)
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
        r = 64
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


@pytest.mark.parametrize("W,M,N,lo,hi", [
    (4, 65, 1, -2, 2), (4, 65, 257, -2, 2), (4, 65, 255, -30000, 30000),
    (8, 66, 513, -50, 50), (4, 131, 700, -3, 3), (8, 97, 1100, -30000, 30000),
    (16, 70, 1025, -5, 5),
])
def test_skew_schedule_matches_oracle(W, M, N, lo, hi):
    rng = np.random.default_rng(W * 1000 + M + N)
    x = rng.integers(lo, hi, size=M).astype(np.int16)
    y = rng.integers(lo, hi, size=N).astype(np.int16)
    assert skew_model(x, y, W) == oracle.sdtw_i64(x, y)
