"""CPU model of the multi-wave (row-band) schedule of the alignment kernel.

One workgroup of P waves aligns one read: the read's M rows are cut into P
bands of consecutive rows (band g: rows [g M / P, (g + 1) M / P)), and wave g
sweeps band g over all reference tiles with the one-wave continuous-skew
schedule (periods of M_g steps, 64K switch steps, boundary column through
the wave's own LDS entries).  Band g's previous row at every tile is the last
row of band g - 1 on that tile (Eq. 1: rows below depend on the rows above
only through that row), handed over through an LDS ring of two tile slots,
plus a ring of four values that carries each tile's last column (the
diagonal that lane 0 needs when it enters the next tile).

Within a period, sub-lane 0 switches at the top of step 0 and every later
sub-lane's switch is issued during the step before its own (after it has
computed its last row on the old tile), except the previous-row reload of
its last group of columns, done at the top of its own step after its right
neighbours have read their edge from them, as the kernel does.  Where the
previous row comes from is also the kernel's: band 0 takes gamma(0, .) = 0
as every other column cleared with the diagonal set to 0, or, streaming,
the resident row's strip and the value left of it from one copy of the
next tile (a single buffer, refilled once every lane has entered the
current tile, when the copy of the current tile has had its last read);
the other bands read the ring.  The reference values of the next tile are held apart
from the last band's staged last rows.

Timing: the workgroup runs global periods G = 0, 1, ... with one barrier
after each; wave g runs its local period p = G - 2g.  Wave g - 1 writes tile
t's last rows during its switch steps of local period t + 1 (global
t + 2g - 1); wave g reads them during its switch steps of local period t
(global t + 2g) and the last column when it enters tile t + 1 (global
t + 2g + 1); tile t + 2 overwrites the slot at global t + 2g + 1, after the
last read of tile t's slot.

The model runs the waves of every global period one after another in a
given order: with both orders the results must equal the oracle's, which
they would not if a slot were written and read in the same global period.
"""
import numpy as np
import pytest

import oracle

INF = 0xFFFFFFFF
L = 64


class Band:
    def __init__(self, g, P, x_rows, ref, W, K, N, shared, acc=None, last=False, gc=8):
        self.g, self.P, self.W, self.K, self.N = g, P, W, K, N
        self.T = L * W
        self.H = W // K
        self.S = L * K
        self.M = len(x_rows)
        assert self.M >= self.S + 1
        self.ref = ref
        self.sh = shared
        self.acc = acc          # resident row (band 0 in streaming mode), written back by the last band
        self.last = last
        S, M = self.S, self.M
        xb = x_rows.astype(np.int64) + 32768
        nent = M + S
        self.bxx = np.array([xb[(k - (S - 1)) % M] for k in range(nent)], np.uint64)
        self.bxy = np.full(nent, INF, np.uint64)
        self.G = min(gc, self.H)  # columns of the deferred last group
        self.stage = np.zeros((L, W), np.uint64)              # finished last rows
        self.ynext = ref[0:self.T].reshape(L, W).copy()       # next tile's reference
        self.y = np.zeros((L, W), np.uint64)
        self.a = np.zeros((L, W), np.uint64)
        self.b = np.zeros((L, W), np.uint64)
        self.dprev = np.full((K, L), INF, np.uint64)
        self.best = np.full(L, INF, np.uint64)
        self.bestj = np.full(L, 2 ** 31 - 1, np.int64)
        self.base = K * (63 - np.arange(L))
        self.nxt = None
        self.accst = None
        self.accleft = None
        if acc is not None and g == 0:
            self.stage_acc(0)

    def stage_acc(self, t):
        T, W = self.T, self.W
        self.accst = self.acc[t * T:(t + 1) * T].reshape(L, W).copy()
        self.accleft = np.array([self.acc[t * T + l * W - 1] if t * T + l * W > 0 else INF
                                 for l in range(L)], np.uint64)

    def entries(self, r):
        return [(self.bxx[self.base + r + (self.K - 1 - h)].copy(),
                 self.bxy[self.base + r + (self.K - 1 - h)].copy()) for h in range(self.K)]

    def sources(self, p):
        """(up source [L, W], dprev of chain 0 [L]) for sub-lanes entering tile p."""
        W = self.W
        if self.g == 0:
            if self.acc is None:  # gamma(0, .) = 0: cleared in registers
                return None, np.zeros(L, np.uint64)
            return self.accst, self.accleft
        ring, edge = self.sh["ring"][self.g - 1], self.sh["edge"][self.g - 1]
        up = ring[p & 1]
        d0 = np.empty(L, np.uint64)
        d0[1:] = up[:-1, W - 1]
        d0[0] = edge[(p - 1) & 3] if p > 0 else INF
        return up, d0

    def step(self, p, r, up, nw, write_b, wrap, sw, src):
        K, H, W, S, M = self.K, self.H, self.W, self.S, self.M
        ent = self.nxt
        self.nxt = self.entries(r + 1)
        lefts = []
        for h in range(K):
            lf = np.empty(L, np.uint64)
            if h == 0:
                lf[1:] = up[:-1, W - 1]
                lf[0] = ent[0][1][0]
            else:
                lf[:] = up[:, h * H - 1]
            lefts.append(lf)
        if sw:
            l, h = r // K, r % K
            upsrc, d0 = src
            if h == K - 1 and l == 63 and not self.last:
                self.sh["edge"][self.g][(p - 1) & 3] = up[l, W - 1]
            if r == 0:  # the period's first switch: all of it, here
                self.switch(p, l, h, up, slice(h * H, (h + 1) * H), src)
                self.dprev[h][l] = self.diag(l, h, src)
            else:       # issued in the previous step but for the last group's
                        # previous row, reloaded after the edges were read
                self.reload(up, l, slice((h + 1) * H - self.G, (h + 1) * H), upsrc)
        for h in range(K):
            ex = ent[h][0]
            diag, lf = self.dprev[h].copy(), lefts[h].copy()
            for w in range(h * H, (h + 1) * H):
                m = np.minimum(np.minimum(up[:, w], diag), lf)
                d = np.abs(ex.astype(np.int64) - self.y[:, w].astype(np.int64)).astype(np.uint64)
                c = (d + m) & 0xFFFFFFFF
                nw[:, w] = c
                diag, lf = up[:, w], c
            self.dprev[h] = lefts[h]
        if write_b:
            self.bxy[r + (M if wrap else 0)] = nw[63, W - 1]
        if sw and r + 1 < S:
            # the next sub-lane has computed its last row on the old tile: its
            # switch is issued now (every group but the last group's previous
            # row, which its right neighbours still read as their edge)
            l, h = (r + 1) // K, (r + 1) % K
            upsrc, d0 = src
            self.switch(p, l, h, nw, slice(h * H, (h + 1) * H - self.G), src,
                        cols=slice(h * H, (h + 1) * H))
            self.dprev[h][l] = self.diag(l, h, src)

    def diag(self, l, h, src):
        """The value left of sub-strip h in the row sub-lane (l, h) enters with."""
        upsrc, d0 = src
        if h == 0:
            return d0[l]
        return 0 if upsrc is None else upsrc[l, h * self.H - 1]

    @staticmethod
    def reload(row, l, cols, upsrc):
        if upsrc is None:  # the odd columns cleared, as the kernel does
            row[l, [c for c in range(cols.start, cols.stop) if c % 2 == 1]] = 0
        else:
            row[l, cols] = upsrc[l, cols]

    def switch(self, p, l, h, row, reload, src, cols=None):
        """Sub-lane (l, h) enters tile p: new reference values, its finished
        row (in `row`) out to the stage (last band) or the ring, the new
        previous row into the columns `reload`."""
        cols = reload if cols is None else cols
        upsrc, _ = src
        if self.last:
            self.stage[l, cols] = row[l, cols]
        else:
            self.sh["ring"][self.g][(p - 1) & 1][l, cols] = row[l, cols]
        self.y[l, cols] = self.ynext[l, cols]
        self.reload(row, l, reload, upsrc)

    def period(self, p, ntiles):
        S, M, T, W = self.S, self.M, self.T, self.W
        a, b = self.a, self.b
        src = self.sources(p)
        self.nxt = self.entries(0)
        for r in range(0, S, 2):
            self.step(p, r, a, b, p > 0 or r == S - 1, r != S - 1, True, src)
            self.step(p, r + 1, b, a, p > 0 or r + 1 == S - 1, r + 1 != S - 1, True, src)
        if p >= 1 and self.last:
            for l in range(L):
                for w in range(W):
                    j = (p - 1) * T + l * W + w
                    if j < self.N and self.stage[l, w] < self.best[l]:
                        self.best[l], self.bestj[l] = self.stage[l, w], j
            if self.acc is not None:
                self.acc[(p - 1) * T:p * T] = self.stage.reshape(-1)
        if p + 1 < ntiles:  # every lane has entered tile p: fetch tile p + 1
            self.ynext[:] = self.ref[(p + 1) * T:(p + 2) * T].reshape(L, W)
            if self.acc is not None and self.g == 0:
                self.stage_acc(p + 1)
        if p == ntiles:
            return
        r = S
        while r + 1 < M:
            self.step(p, r, a, b, True, False, False, None)
            self.step(p, r + 1, b, a, True, False, False, None)
            r += 2
        if r < M:
            self.step(p, r, a, b, True, False, False, None)
            a[:] = b


def band_model(x, yref, W, K, P, order=1, acc=None):
    """Run the P-band schedule; returns (cost, end) and, in streaming mode
    (acc = gamma(m_old, .) padded to whole tiles), the written-back row."""
    T = L * W
    M, N = len(x), len(yref)
    ntiles = (N + T - 1) // T
    ref = np.zeros(ntiles * T + T, np.uint64)
    ref[:N] = yref.astype(np.int64) + 32768
    shared = {"ring": np.zeros((P, 2, L, W), np.uint64), "edge": np.zeros((P, 4), np.uint64)}
    cuts = [(g * M) // P for g in range(P + 1)]
    bands = [Band(g, P, x[cuts[g]:cuts[g + 1]], ref, W, K, N, shared, acc, g == P - 1)
             for g in range(P)]
    for G in range(ntiles + 1 + 2 * (P - 1)):
        for g in (range(P) if order > 0 else range(P - 1, -1, -1)):
            p = G - 2 * g
            if 0 <= p <= ntiles:
                bands[g].period(p, ntiles)
    lb = bands[-1]
    i = np.lexsort((lb.bestj, lb.best))[0]
    return int(lb.best[i]), int(lb.bestj[i])


CASES = [
    # W, K, P, M, N, value range
    (4, 1, 2, 130, 1, 3), (4, 1, 2, 131, 700, 3), (4, 1, 3, 200, 1100, 30000),
    (4, 1, 4, 260, 1025, 5), (4, 1, 4, 263, 300, 30000), (8, 1, 2, 140, 1500, 40),
    (4, 2, 2, 258, 600, 3), (8, 2, 2, 300, 1030, 30000),
]


@pytest.mark.parametrize("W,K,P,M,N,hi", CASES)
@pytest.mark.parametrize("order", [1, -1])
def test_band_schedule_matches_oracle(W, K, P, M, N, hi, order):
    rng = np.random.default_rng(W * 1000 + K * 100 + P * 10 + M + N)
    x = rng.integers(-hi, hi, size=M).astype(np.int16)
    y = rng.integers(-hi, hi, size=N).astype(np.int16)
    assert band_model(x, y, W, K, P, order) == oracle.sdtw_i64(x, y)


@pytest.mark.parametrize("W,K,P,m_old,M,N", [(4, 1, 2, 50, 130, 700), (4, 1, 3, 1, 195, 1025),
                                             (8, 2, 2, 300, 258, 900)])
@pytest.mark.parametrize("order", [1, -1])
def test_band_schedule_streaming_matches_oracle(W, K, P, m_old, M, N, order):
    rng = np.random.default_rng(m_old + M + N + P)
    x = rng.integers(-40, 40, size=m_old + M).astype(np.int16)
    y = rng.integers(-40, 40, size=N).astype(np.int16)
    T = L * W
    _, _, row = oracle.sdtw_i64(x[:m_old], y, lastrow=True)
    acc = np.zeros(((N + T - 1) // T) * T + T, np.uint64)
    acc[:N] = row.astype(np.uint64)
    cost, end = band_model(x[m_old:], y, W, K, P, order, acc)
    wc, we, wrow = oracle.sdtw_i64(x, y, lastrow=True)
    assert (cost, end) == (wc, we)
    assert np.array_equal(acc[:N].astype(np.int64), wrow)


def test_ring_slots_are_never_read_and_written_in_one_global_period():
    # writer (wave g - 1) writes tile t at global period t + 2g - 1 into slot
    # t & 1 and its last column into edge slot t & 3; the reader (wave g)
    # reads the slot at t + 2g and the edge at t + 2g + 1
    for g in (1, 2, 3):
        for t in range(12):
            w_slot = t + 2 * g - 1
            r_slot, r_edge = t + 2 * g, t + 2 * g + 1
            assert w_slot < r_slot and w_slot < r_edge
            # the next writes into the same slots come strictly later
            assert (t + 2) + 2 * g - 1 > r_slot
            assert (t + 4) + 2 * g - 1 > r_edge


@pytest.mark.parametrize("W,K,P,M,g", [(4, 1, 2, 140, 1), (4, 1, 3, 200, 1), (4, 1, 3, 200, 2),
                                       (4, 1, 4, 270, 3), (8, 2, 2, 270, 1)])
def test_band_boundary_diagonal_on_exact_substring(W, K, P, M, g):
    # x is an exact substring of y whose zero-cost diagonal path crosses from
    # band g - 1 into band g exactly at a tile boundary, so the diagonal value
    # lane 0 takes from the previous tile's last column decides the result
    T = L * W
    rng = np.random.default_rng(M + g)
    y = rng.permutation(np.arange(-20000, 20000, 7))[:5 * T].astype(np.int16)
    r0 = (g * M) // P
    s = 2 * T - r0
    x = y[s:s + M].copy()
    want = oracle.sdtw_i64(x, y)
    assert want == (0, s + M - 1)
    assert band_model(x, y, W, K, P) == want
