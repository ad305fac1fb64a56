"""GPU streaming extension against the oracle.

A read that arrives in chunks is normalised with the statistics of its first
chunk; extending its resident row chunk by chunk must give exactly what the
oracle gives on the concatenated prefix (row i of Eq. 1 depends on X[1..i]
only): the same cost and end after every chunk, and the same last row.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

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


@pytest.fixture(scope="module")
def prepared():
    w = synth.workload(1, nq=16)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    return w, z, codes


def chunked_reads(w, plans, seed=0):
    """Raw pA events of reads cut into chunks; each chunk scaled with the
    statistics of its read's first chunk (oracle)."""
    rng = np.random.default_rng(seed)
    reads = []
    for r, sizes in enumerate(plans):
        total = int(sum(sizes))
        if r % 2 == 0:
            sim = synth.simulate_reads(w.genome, w.table, [total], 1.0, seed + r)
        else:
            sim = synth.simulate_reads(w.genome, w.table, [total], 0.0, seed + r)
        raw = sim.values
        cuts = np.concatenate([[0], np.cumsum(sizes)])
        mean, sdv = oracle.zstats(raw[:cuts[1]])
        z = oracle.zapply(raw, mean, sdv)
        codes, _ = oracle.quantize(z, 64.0)
        reads.append((raw, z, codes, cuts))
    return reads


def run_rounds(dev, ref_np, reads, dt):
    """Extend every stream round by round (one batched call per round) and
    check each result against the oracle on the concatenated prefix."""
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    streams = [sd.Stream(ref) for _ in reads]
    nrounds = max(len(c) - 1 for _, _, _, c in reads)
    got_all = []
    for k in range(nrounds):
        live = [i for i, (_, _, _, c) in enumerate(reads) if k < len(c) - 1]
        vals = [(reads[i][2] if dt == sd.I16 else reads[i][1])[reads[i][3][k]:reads[i][3][k + 1]]
                for i in live]
        q, offs = synth.csr(vals)
        q = q.astype(np.int16 if dt == sd.I16 else np.float32)
        note(f"round {k}: {len(live)} streams, chunk lengths {np.diff(offs).tolist()}")
        cost, end = sd.stream_extend([streams[i] for i in live], torch.from_numpy(q).to(dev),
                                     offs)
        torch.cuda.synchronize()
        cost, end = cost.cpu().numpy(), end.cpu().numpy()
        for t, i in enumerate(live):
            cut = reads[i][3][k + 1]
            prefix = (reads[i][2] if dt == sd.I16 else reads[i][1])[:cut]
            if dt == sd.I16:
                wc, we, lr = oracle.sdtw_i64(prefix, ref_np, lastrow=True)
                assert (int(cost[t]), int(end[t])) == (wc, we), (i, k)
            else:
                wc, we, lr = oracle.sdtw_f32(prefix, ref_np, lastrow=True)
                assert (np.float32(cost[t]), int(end[t])) == (wc, we), (i, k)
            assert streams[i].rows == cut
            row = streams[i].copy_row().cpu().numpy()
            torch.cuda.synchronize()
            if dt == sd.I16:
                assert np.array_equal(row.astype(np.int64), lr), (i, k)
            else:
                assert np.array_equal(row.view(np.uint32), lr.view(np.uint32)), (i, k)
            got_all.append((i, k, int(end[t]), float(cost[t])))
    for s in streams:
        s.close()
    ref.close()
    return got_all


PLANS = [[400, 400, 400], [70, 30, 300], [1, 64, 65, 200], [250], [65, 65, 65, 65, 65],
         [129, 1, 2], [300, 64]]


@pytest.mark.parametrize("dt", ["i16", "f32"])
@pytest.mark.parametrize("strip,bands", [(0, 0), (16, 1), (16, 2), (16, 3), (16, 4), (32, 1),
                                         (32, 2), (32, 3), (32, 4)])
def test_extend_equals_from_scratch(dev, prepared, dt, strip, bands):
    w, z, codes = prepared
    reads = chunked_reads(w, PLANS)
    sd.set_stream_config(strip, bands)
    try:
        run_rounds(dev, codes if dt == "i16" else z, reads, sd.I16 if dt == "i16" else sd.F32)
    finally:
        sd.set_stream_config(0, 0)


@pytest.mark.parametrize("strip,bands", [(16, 1), (16, 4), (32, 4)])
def test_extend_diagonal_at_chunk_and_band_boundaries(dev, strip, bands):
    # a read that is an exact substring of the reference, cut into chunks so
    # that its zero-cost diagonal crosses the first chunk boundary exactly at
    # a tile boundary (column 2T) and, with four bands, the boundary between
    # bands 0 and 1 of the third chunk (2016 rows, bands of 504) at column 3T
    T = 64 * (strip or 16)
    rng = np.random.default_rng(17 + bands + strip)
    ref = rng.permutation(np.arange(-30000, 30000, 4))[:6 * T].astype(np.int16)
    s = 2 * T - 300
    c2 = T - 504
    x = ref[s:s + 300 + c2 + 2016].copy()
    assert s + 300 + c2 + 504 == 3 * T
    reads = [(None, None, x, np.array([0, 300, 300 + c2, x.size]))]
    sd.set_stream_config(strip, bands)
    try:
        got = run_rounds(dev, ref, reads, sd.I16)
    finally:
        sd.set_stream_config(0, 0)
    assert [(e, c) for (_, _, e, c) in got] == [(s + 299, 0.0), (s + 299 + c2, 0.0),
                                                (s + x.size - 1, 0.0)]


@pytest.mark.parametrize("dt", ["i16", "f32"])
def test_best_two_matches_oracle(dev, prepared, dt):
    # best and runner-up ends of resident rows after ragged extensions, for
    # windows from 0 to beyond the row (no runner-up)
    w, z, codes = prepared
    ref_np = codes if dt == "i16" else z
    reads = chunked_reads(w, PLANS[:5], seed=21)
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    streams = [sd.Stream(ref) for _ in reads]
    vals = [(r[2] if dt == "i16" else r[1]) for r in reads]
    q, offs = synth.csr(vals)
    q = q.astype(np.int16 if dt == "i16" else np.float32)
    sd.stream_extend(streams, torch.from_numpy(q).to(dev), offs)
    for window in (0, 3, 250, 40000, ref_np.size):
        bc, be, sc, se = [t.cpu().numpy() for t in sd.stream_best_two(streams, window)]
        torch.cuda.synchronize()
        for i, v in enumerate(vals):
            if dt == "i16":
                _, _, row = oracle.sdtw_i64(v, ref_np, lastrow=True)
                want = oracle.best_two(row, window)
                got = (int(bc[i]), int(be[i]),
                       float("inf") if se[i] < 0 else int(sc[i]), int(se[i]))
            else:
                _, _, row = oracle.sdtw_f32(v, ref_np, lastrow=True)
                want = oracle.best_two(row, window)
                want = (np.float32(want[0]), want[1], np.float32(want[2]), want[3])
                got = (np.float32(bc[i]), int(be[i]), np.float32(sc[i]), int(se[i]))
            assert got == tuple(want), (i, window)
            if se[i] < 0:
                assert sc[i] == (np.iinfo(np.int32).max if dt == "i16" else np.inf)
    for st in streams:
        st.close()
    ref.close()


@pytest.mark.parametrize("dt", ["i16", "f32"])
def test_best_two_segment_edges(dev, dt):
    # a one-event read makes the last row |x - y_j| exactly, so the row can
    # be planted: minima on both sides of the first-pass segment edges
    # (16,384 columns), ties across an edge, and windows that end exactly on
    # a planted column or one past it
    n = 3 * 16384 + 77
    ref_np = np.full(n, 100, np.int16)
    for c, v in ((16383, 5), (16384, 5), (16390, 6), (32767, 7), (32768, 7), (40000, 8),
                 (0, 9), (n - 1, 10)):
        ref_np[c] = v
    x = np.zeros(1, np.int16)
    if dt == "f32":
        ref_np, x = ref_np.astype(np.float32), x.astype(np.float32)
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    st = sd.Stream(ref)
    sd.stream_extend([st], torch.from_numpy(x).to(dev), np.array([0, 1], np.int64))
    row = np.abs(ref_np.astype(np.int64))
    for window in (0, 1, 6, 7, 16382, 16383, 16384, 16385, 23616, 23617, 32844, 32845, n):
        bc, be, sc, se = [t.cpu().numpy() for t in sd.stream_best_two([st], window)]
        want = oracle.best_two(row, window)
        got = (int(bc[0]), int(be[0]), float("inf") if se[0] < 0 else int(sc[0]), int(se[0]))
        assert got == (int(want[0]), want[1], want[2] if want[3] < 0 else int(want[2]),
                       want[3]), window
    st.close()
    ref.close()


def test_extend_ragged_reference(dev):
    rng = np.random.default_rng(4)
    ref = rng.integers(-3000, 3000, size=3001).astype(np.int16)
    reads = []
    for sizes in ([100, 200, 5], [1, 1, 1], [64, 64], [70, 2000]):
        total = int(sum(sizes))
        codes = rng.integers(-3000, 3000, size=total).astype(np.int16)
        reads.append((None, None, codes, np.concatenate([[0], np.cumsum(sizes)])))
    run_rounds(dev, ref, reads, sd.I16)


def test_alone_equals_mixed(dev, prepared):
    w, z, codes = prepared
    reads = chunked_reads(w, PLANS, seed=10)
    mixed = run_rounds(dev, codes, reads, sd.I16)
    alone = []
    for i in range(len(reads)):
        alone += [(i, k, e, c) for (_, k, e, c) in run_rounds(dev, codes, [reads[i]], sd.I16)]
    assert sorted(mixed) == sorted(alone)


def test_prepare_queries_with_fixed_statistics(dev):
    w = synth.workload(1, nq=20)
    raw = w.reads.values
    offs = w.reads.offsets
    stats = np.array([oracle.zstats(raw[offs[r]:offs[r] + 100]) for r in range(20)])
    z, codes, nsat, used = sd.prepare_queries_ex(torch.from_numpy(raw).to(dev),
                                                 torch.from_numpy(offs).to(dev), 64.0,
                                                 torch.from_numpy(stats).to(dev))
    torch.cuda.synchronize()
    want = np.concatenate([oracle.zapply(raw[offs[r]:offs[r + 1]], *stats[r])
                           for r in range(20)])
    assert np.array_equal(z.cpu().numpy().view(np.uint32), want.view(np.uint32))
    assert np.array_equal(codes.cpu().numpy(), oracle.quantize(want, 64.0)[0])
    assert np.array_equal(used.cpu().numpy(), stats)
    # without stats_in the statistics are each read's own (oracle.zstats)
    _, _, _, own = sd.prepare_queries_ex(torch.from_numpy(raw).to(dev),
                                         torch.from_numpy(offs).to(dev), 64.0)
    torch.cuda.synchronize()
    assert np.array_equal(own.cpu().numpy(),
                          np.array([oracle.zstats(raw[offs[r]:offs[r + 1]]) for r in range(20)]))


def test_budget_and_state_errors(dev, prepared):
    w, z, codes = prepared
    ref = sd.Reference(torch.from_numpy(codes).to(dev))
    other = sd.Reference(torch.from_numpy(codes[:5000].copy()).to(dev))
    budget0 = sd.row_budget_info()[0]
    try:
        row_bytes = 4 * (((codes.size + 2047) // 2048) * 2048 + 2048)
        sd.set_row_budget(row_bytes * 2)
        a, b = sd.Stream(ref), sd.Stream(ref)
        with pytest.raises(sd.SdtwError) as ei:
            sd.Stream(ref)
        assert ei.value.code == "EBUDGET"
        with pytest.raises(sd.SdtwError) as ei:
            a.copy_row()
        assert ei.value.code == "ESTATE"
        with pytest.raises(sd.SdtwError) as ei:
            ref.close()  # streams are open on it
        assert ei.value.code == "ESTATE"
        q = torch.zeros(100, dtype=torch.int16, device=dev)
        with pytest.raises(sd.SdtwError) as ei:
            sd.stream_extend([a, a], q, [0, 50, 100])
        assert ei.value.code == "EINVAL"
        b.close()
        c = sd.Stream(ref)  # room again after a close
        cost, end = sd.stream_extend([a, c], q, [0, 50, 100])
        torch.cuda.synchronize()
        assert a.rows == 50 and c.rows == 50
        o = None
        sd.set_row_budget(row_bytes * 3)
        o = sd.Stream(other)
        with pytest.raises(sd.SdtwError) as ei:
            sd.stream_extend([a, o], q, [0, 50, 100])  # different references
        assert ei.value.code == "EINVAL"
        for s in (a, c, o):
            s.close()
        assert sd.row_budget_info()[1] == 0 and sd.row_budget_info()[2] > 0
        sd.row_pool_trim()
        assert sd.row_budget_info()[2] == 0  # cached rows freed
    finally:
        sd.set_row_budget(budget0)
    other.close()
    ref.close()


def _wide_rounds(dev, ref_np, chunks, ways, cols):
    """One stream extended chunk by chunk, each chunk by the whole-device scan
    ("wide") or the batched kernel ("batch"); after every chunk the cost, the
    end and the whole resident row equal the oracle's on the prefix."""
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    s = sd.Stream(ref)
    done = []
    try:
        for k, (ck, way) in enumerate(zip(chunks, ways)):
            note(f"wide extension: chunk {k} ({ck.size} rows) by {way}, cols={cols}, "
                 f"N={ref_np.size}")
            q = torch.from_numpy(ck).to(dev)
            if way == "wide":
                cost, end = sd.stream_extend_wide(s, q, cols)
            else:
                cost, end = sd.stream_extend([s], q, np.array([0, ck.size], np.int64))
            row = s.copy_row()
            torch.cuda.synchronize()
            done.append(ck)
            want_c, want_e, want_row = oracle.sdtw_i64(np.concatenate(done), ref_np,
                                                       lastrow=True)
            assert (int(cost.item()), int(end.item())) == (want_c, want_e), (k, way)
            assert np.array_equal(row.cpu().numpy().astype(np.int64), want_row), (k, way)
            assert s.rows == sum(c.size for c in done)
    finally:
        torch.cuda.synchronize()
        s.close()
        ref.close()


@pytest.mark.parametrize("cols", [0, 8, 16, 32, 64])
def test_extend_wide_matches_oracle(dev, cols):
    # three chunks over one or many tiles and a ragged last tile; the
    # first starts from the free-start row, the others from the resident row
    rng = np.random.default_rng(40 + cols)
    ref_np = rng.integers(-3000, 3000, size=37_001).astype(np.int16)
    chunks = [rng.integers(-3000, 3000, size=m).astype(np.int16) for m in (150, 1, 97)]
    _wide_rounds(dev, ref_np, chunks, ["wide"] * 3, cols)


def test_extend_wide_and_batched_take_turns(dev):
    # one resident row format: the two paths extend the same stream in turn
    rng = np.random.default_rng(41)
    ref_np = rng.integers(-3000, 3000, size=20_000).astype(np.int16)
    chunks = [rng.integers(-3000, 3000, size=m).astype(np.int16) for m in (200, 130, 300, 70)]
    _wide_rounds(dev, ref_np, chunks, ["batch", "wide", "batch", "wide"], 16)


def test_extend_wide_more_tiles_than_resident(dev):
    # 5,000,000 columns at 8 per thread: 2,442 tiles, more than the device
    # holds at once, so later tiles start after earlier ones have written
    # their new rows back (each tile's left value is taken aside first)
    rng = np.random.default_rng(42)
    ref_np = rng.integers(-3000, 3000, size=5_000_000).astype(np.int16)
    chunks = [rng.integers(-3000, 3000, size=m).astype(np.int16) for m in (60, 45)]
    _wide_rounds(dev, ref_np, chunks, ["wide", "wide"], 8)


def test_extend_wide_rejections(dev):
    rng = np.random.default_rng(43)
    ref = sd.Reference(torch.from_numpy(rng.integers(-99, 99, size=3000).astype(np.int16))
                       .to(dev))
    s = sd.Stream(ref)
    try:
        big = torch.from_numpy(rng.integers(-99, 99, size=4000).astype(np.int16)).to(dev)
        sd.stream_extend_wide(s, big[:4000])
        with pytest.raises(sd.SdtwError) as e:  # 4,000 + 97 rows > 4,096
            sd.stream_extend_wide(s, big[:97])
        assert e.value.code == "EINVAL"
        with pytest.raises(sd.SdtwError):
            sd.stream_extend_wide(s, big[:5], cols=12)
        assert s.rows == 4000
    finally:
        torch.cuda.synchronize()
        s.close()
        ref.close()
    fref = sd.Reference(torch.from_numpy(rng.normal(size=3000).astype(np.float32)).to(dev))
    fs = sd.Stream(fref)
    try:
        with pytest.raises(sd.SdtwError) as e:
            sd.stream_extend_wide(fs, torch.zeros(10, dtype=torch.int16, device=dev))
        assert e.value.code == "EINVAL"
    finally:
        fs.close()
        fref.close()


def test_long_reference_batches_at_once(dev):
    # two batched extensions of 256 resident rows each against a reference of
    # more than 2^20 columns (strip 32, four bands), issued at once on two HIP
    # streams so that their workgroups share CUs (together they cover more
    # than half the device: no LDS reservation), give what the same
    # extensions give one after another, and sampled rows match the oracle
    budget0 = sd.row_budget_info()[0]
    sd.set_row_budget(16 << 30)  # 512 rows of about 4 MB at a time
    rng = np.random.default_rng(23)
    n = (1 << 20) + 12345
    ref_np = rng.integers(-3000, 3000, size=n).astype(np.int16)
    ref = sd.Reference(torch.from_numpy(ref_np).to(dev))
    k, m = 256, 400
    chunks = [rng.integers(-3000, 3000, size=(2, 2 * k, m)).astype(np.int16)]
    offs = np.arange(k + 1, dtype=np.int64) * m
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]

    def run(together):
        st = [sd.Stream(ref) for _ in range(2 * k)]
        res = []
        for c in range(2):
            qa = torch.from_numpy(chunks[0][c, :k].reshape(-1)).to(dev)
            qb = torch.from_numpy(chunks[0][c, k:].reshape(-1)).to(dev)
            torch.cuda.synchronize()
            ca, ea = sd.stream_extend(st[:k], qa, offs, stream=hs[0])
            if not together:
                hs[0].synchronize()
            cb, eb = sd.stream_extend(st[k:], qb, offs, stream=hs[1])
            torch.cuda.synchronize()
            res.append((ca.cpu().numpy(), ea.cpu().numpy(), cb.cpu().numpy(), eb.cpu().numpy()))
        for s in st:
            s.close()
        return res

    note("two long-reference batches one after another, then at once")
    apart = run(False)
    together = run(True)
    for a, b in zip(apart, together):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    for i in (0, k - 1, k, 2 * k - 1):
        prefix = np.concatenate([chunks[0][0, i], chunks[0][1, i]])
        wc, we = oracle.sdtw_i64(prefix, ref_np)
        half = 0 if i < k else 1
        t = i if i < k else i - k
        assert (int(together[1][2 * half][t]), int(together[1][2 * half + 1][t])) == (wc, we), i
    ref.close()
    sd.set_row_budget(budget0)
