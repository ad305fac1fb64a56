"""GPU parity: the HIP path against the CPU oracle, element by element.

Bars: the int16 path is bit-exact against the exact integer oracle (cost and
end); the float32 path is bit-exact against the float32-sequenced oracle and
its cost lies within 1e-5 relative of the float64 oracle, whose last row must
also accept the GPU's end (gamma64(M, end) <= cost64 * (1 + 1e-5)).
Inputs are seeded and synthetic (synth) and prepared by the oracle, so the
GPU and the oracle see identical arrays.
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
def small_ref():
    w = synth.workload(1, nq=64)
    z, codes, nsat = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    return w, z, codes, qz, qc


def gpu_batch(dev, ref_np, q_np, offs, dtype, strip=0, waves=0, chains=0, bands=0,
              band_rows=-1):
    ref = sd.Reference(torch.from_numpy(np.ascontiguousarray(ref_np)).to(dev))
    plan = sd.Plan(offs, dtype)
    if strip or waves or chains or bands or band_rows >= 0:
        plan.set_config(strip, chains, waves, bands, band_rows)
    cost, end = sd.align_batch(ref, plan, torch.from_numpy(np.ascontiguousarray(q_np)).to(dev))
    torch.cuda.synchronize()
    out = cost.cpu().numpy(), end.cpu().numpy()
    plan.close()
    ref.close()
    return out


def check_i16(got, q, offs, ref, index=None):
    want_c, want_e, _ = oracle.batch(oracle.I64, q, offs, ref, index=index)
    gc, ge = got
    if index is not None:
        gc, ge = gc[index], ge[index]
    bad = np.nonzero((gc.astype(np.int64) != want_c.astype(np.int64)) | (ge != want_e))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first {bad[:5]}: " \
        f"gpu {gc[bad[:5]]},{ge[bad[:5]]} oracle {want_c[bad[:5]]},{want_e[bad[:5]]}"


def check_f32(got, q, offs, ref, index=None, f64=True):
    want_c, want_e, _ = oracle.batch(oracle.F32, q, offs, ref, index=index)
    gc, ge = got
    if index is not None:
        gc, ge = gc[index], ge[index]
    bad = np.nonzero((gc.astype(np.float64) != want_c) | (ge != want_e))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first {bad[:5]}: " \
        f"gpu {gc[bad[:5]]},{ge[bad[:5]]} oracle {want_c[bad[:5]]},{want_e[bad[:5]]}"
    if f64:
        rows = range(offs.size - 1) if index is None else index
        for t, r in enumerate(rows):
            x = q[offs[r]:offs[r + 1]]
            c64, e64, lr = oracle.sdtw_f64(x, ref, lastrow=True)
            assert abs(float(gc[t]) - c64) <= 1e-5 * max(c64, 1e-30), (r, gc[t], c64)
            assert lr[ge[t]] <= c64 * (1 + 1e-5) + 1e-30, (r, ge[t], e64)


# ---------------------------------------------------------------------------


def test_single_read_one_per_launch(dev, small_ref):
    w, z, codes, qz, qc = small_ref
    offs = w.reads.offsets
    for r in (0, 1):
        a, b = offs[r], offs[r + 1]
        for dt, refv, qv in ((sd.I16, codes, qc), (sd.F32, z, qz)):
            note(f"align_one read {r} dtype {dt} M={b - a} N={refv.size}")
            ref = sd.Reference(torch.from_numpy(refv).to(dev))
            cost, end = sd.align_one(ref, torch.from_numpy(qv[a:b].copy()).to(dev))
            torch.cuda.synchronize()
            if dt == sd.I16:
                want = oracle.sdtw_i64(qv[a:b], refv)
                assert (int(cost.item()), int(end.item())) == want
            else:
                want = oracle.sdtw_f32(qv[a:b], refv)
                assert (np.float32(cost.item()), int(end.item())) == (want[0], want[1])
            ref.close()


def test_batch_64_reads_small_reference(dev, small_ref):
    w, z, codes, qz, qc = small_ref
    offs = w.reads.offsets
    note("batch 64 x M=250 int16")
    check_i16(gpu_batch(dev, codes, qc, offs, sd.I16), qc, offs, codes)
    note("batch 64 x M=250 float32")
    check_f32(gpu_batch(dev, z, qz, offs, sd.F32), qz, offs, z,
              index=np.arange(0, 64, 8))


@pytest.mark.parametrize("strip,chains", [(8, 1), (8, 2), (16, 1), (16, 2), (16, 4), (32, 1),
                                          (32, 2), (32, 4)])
@pytest.mark.parametrize("waves", [1, 3, 16])
def test_schedule_invariance(dev, small_ref, strip, chains, waves):
    w, z, codes, qz, qc = small_ref
    offs = w.reads.offsets[:17]
    note(f"schedule strip={strip} chains={chains} waves={waves}")
    check_i16(gpu_batch(dev, codes, qc, offs, sd.I16, strip, waves, chains), qc, offs, codes)
    check_f32(gpu_batch(dev, z, qz, offs, sd.F32, strip, waves, chains), qz, offs, z, f64=False)


def _ragged_case(seed, Ms, N, lo=-3000, hi=3000):
    rng = np.random.default_rng(seed)
    ref = rng.integers(lo, hi, size=N).astype(np.int16)
    qs = [rng.integers(lo, hi, size=m).astype(np.int16) for m in Ms]
    vals, offs = synth.csr(qs)
    return ref, vals.astype(np.int16), offs


@pytest.mark.parametrize("strip,chains,bands,waves", [
    (16, 1, 2, 2), (16, 1, 2, 8), (16, 1, 4, 4), (16, 1, 4, 16), (16, 2, 2, 4), (16, 2, 4, 8),
    (32, 1, 2, 4), (32, 1, 4, 8), (16, 1, 3, 3), (16, 1, 3, 12), (32, 1, 3, 6),
    (32, 2, 2, 4), (32, 2, 2, 8)])
def test_band_schedule_invariance(dev, strip, chains, bands, waves):
    # row bands (several waves per read): reads whose band count ranges from
    # 1 to 4, band heights at the minimum and ragged, several tiles and a
    # ragged tail, few and many workgroups per compute unit
    Ms = [65, 129, 130, 131, 200, 259, 260, 261, 263, 400, 517, 1000, 2049, 4096]
    ref, q, offs = _ragged_case(bands * 10 + chains + strip, Ms, 5000)
    note(f"strip={strip} bands={bands} chains={chains} waves={waves} Ms={Ms}")
    check_i16(gpu_batch(dev, ref, q, offs, sd.I16, strip, waves, chains, bands), q, offs, ref)
    rng = np.random.default_rng(bands + chains)
    zref = rng.normal(size=3001).astype(np.float32)
    zq, zoffs = synth.csr([rng.normal(size=m).astype(np.float32) for m in Ms[:12]])
    check_f32(gpu_batch(dev, zref, zq.astype(np.float32), zoffs, sd.F32, strip, waves, chains,
                        bands), zq.astype(np.float32), zoffs, zref)


@pytest.mark.parametrize("per_cu,extra", [(1, 0), (1, 37), (2, -5)])
def test_band_pulls_from_both_ends(dev, per_cu, extra):
    # two-wave workgroups (per_cu of them on every compute unit): with no more
    # reads than workgroups half of them take their read from the back of the
    # longest-first list, chosen by the SIMD their first wave runs on; with
    # more, every pull takes the front; either way every read exactly once
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = per_cu * cus + extra
    rng = np.random.default_rng(n)
    Ms = [int(m) for m in rng.integers(130, 601, size=n)]
    ref, q, offs = _ragged_case(n, Ms, 2500)
    note(f"both ends: {n} reads, {per_cu} two-band workgroups per CU on {cus} CUs")
    check_i16(gpu_batch(dev, ref, q, offs, sd.I16, 32, 2 * per_cu, 1, 2), q, offs, ref)


@pytest.mark.parametrize("strip,bands,band_rows", [(16, 4, 100), (32, 4, 125), (32, 3, 70),
                                                   (16, 2, 300)])
def test_band_row_targets(dev, strip, bands, band_rows):
    # a target band height gives reads of different lengths different band
    # counts (1 to `bands`) in one launch
    Ms = [65, 100, 130, 150, 199, 260, 300, 333, 400, 450, 500, 777, 1500]
    ref, q, offs = _ragged_case(strip + bands + band_rows, Ms, 4100)
    note(f"band rows strip={strip} bands={bands} target={band_rows}")
    check_i16(gpu_batch(dev, ref, q, offs, sd.I16, strip, 4 * bands, 1, bands, band_rows),
              q, offs, ref)


@pytest.mark.parametrize("strip,chains,bands", [(16, 1, 2), (16, 1, 4), (16, 2, 2), (16, 2, 4),
                                                (32, 1, 2), (32, 1, 4), (16, 1, 3),
                                                (32, 1, 3), (32, 2, 2)])
def test_band_boundary_diagonal_on_exact_substrings(dev, strip, chains, bands):
    # each read is an exact substring of the reference whose zero-cost
    # diagonal crosses from band g - 1 into band g exactly at a tile
    # boundary, so the diagonal handed over with the previous tile's last
    # column decides the result (cost 0, end s + M - 1)
    T = 64 * strip
    rng = np.random.default_rng(5 + bands + chains + strip)
    ref = rng.permutation(np.arange(-32000, 32000, 5))[:6 * T].astype(np.int16)
    S1 = 64 * chains + 1
    qs, want = [], []
    for M in (bands * S1, bands * S1 + 37, 4 * bands * S1 + 3):
        pe = min(bands, M // S1)
        for g in range(1, pe):
            s = 2 * T - (g * M) // pe
            qs.append(ref[s:s + M].copy())
            want.append((0, s + M - 1))
    q, offs = synth.csr(qs)
    q = q.astype(np.int16)
    note(f"diagonal bands={bands} chains={chains} reads={len(qs)}")
    got = gpu_batch(dev, ref, q, offs, sd.I16, strip, 4 * bands, chains, bands)
    assert list(zip(got[0].tolist(), got[1].tolist())) == want
    check_i16(got, q, offs, ref)


@pytest.mark.parametrize("N", [1, 7, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 2047, 2048,
                               2049, 5000])
def test_edge_lengths_int16(dev, N):
    Ms = [1, 2, 5, 33, 63, 64, 65, 66, 100, 127, 128, 129, 130, 250, 256, 257, 258, 700]
    ref, q, offs = _ragged_case(N, Ms, N)
    note(f"edge int16 N={N} Ms={Ms}")
    for strip, chains in ((8, 2), (16, 1), (16, 2), (16, 4), (32, 2), (32, 4)):
        check_i16(gpu_batch(dev, ref, q, offs, sd.I16, strip, 2, chains), q, offs, ref)


@pytest.mark.parametrize("N", [1, 65, 1025, 3001])
def test_edge_lengths_float32(dev, N):
    Ms = [1, 3, 63, 64, 65, 129, 200, 257, 1500]
    rng = np.random.default_rng(N + 7)
    ref = rng.normal(size=N).astype(np.float32)
    qs = [rng.normal(size=m).astype(np.float32) for m in Ms]
    q, offs = synth.csr(qs)
    q = q.astype(np.float32)
    note(f"edge float32 N={N}")
    check_f32(gpu_batch(dev, ref, q, offs, sd.F32, 16, 2), q, offs, ref)


def test_ties_constant_reference_and_extremes(dev):
    # constant reference: every column ties, the first (end 0) must win
    ref = np.full(3000, 17, np.int16)
    qs = [np.full(m, v, np.int16) for m, v in ((70, 17), (300, -5), (64, 17), (10, 3))]
    q, offs = synth.csr(qs)
    q = q.astype(np.int16)
    got = gpu_batch(dev, ref, q, offs, sd.I16)
    assert got[1].tolist() == [0, 0, 0, 0]
    assert got[0].tolist() == [0, 300 * 22, 0, 10 * 14]
    check_i16(got, q, offs, ref)
    # int16 extremes: |x - y| up to 65535 per cell, costs near 2^31 stay exact
    rng = np.random.default_rng(99)
    ref = rng.choice(np.array([-32768, 32767], np.int16), size=4000)
    qs = [rng.choice(np.array([-32768, 32767], np.int16), size=m) for m in (64, 129, 2000, 4096)]
    q, offs = synth.csr(qs)
    q = q.astype(np.int16)
    note("extremes int16")
    check_i16(gpu_batch(dev, ref, q, offs, sd.I16), q, offs, ref)
    qs = [np.full(m, -32768, np.int16) for m in (4096, 100)]
    q, offs = synth.csr(qs)
    q = q.astype(np.int16)
    ref = np.full(50, 32767, np.int16)
    got = gpu_batch(dev, ref, q, offs, sd.I16)
    assert got[0].tolist() == [4096 * 65535, 100 * 65535]


def test_query_longer_than_reference(dev):
    ref, q, offs = _ragged_case(5, [400, 64, 90], 37)
    check_i16(gpu_batch(dev, ref, q, offs, sd.I16), q, offs, ref)


def test_exact_substring_zero_cost(dev, small_ref):
    w, z, codes, qz, qc = small_ref
    rng = np.random.default_rng(1)
    starts = rng.integers(0, z.size - 300, size=8)
    Ms = rng.integers(64, 300, size=8)
    qs = [z[s:s + m].copy() for s, m in zip(starts, Ms)]
    q, offs = synth.csr(qs)
    q = q.astype(np.float32)
    c, e = gpu_batch(dev, z, q, offs, sd.F32)
    assert np.all(c == 0.0)
    assert np.all(e <= starts + Ms - 1)
    check_f32((c, e), q, offs, z, f64=False)


def test_alone_equals_in_batch(dev, small_ref):
    w, z, codes, qz, qc = small_ref
    offs = w.reads.offsets[:9]
    batch = gpu_batch(dev, codes, qc, offs, sd.I16)
    ref = sd.Reference(torch.from_numpy(codes).to(dev))
    for r in range(8):
        cost, end = sd.align_one(ref, torch.from_numpy(qc[offs[r]:offs[r + 1]].copy()).to(dev))
        torch.cuda.synchronize()
        assert (int(cost.item()), int(end.item())) == (int(batch[0][r]), int(batch[1][r]))
    ref.close()


def test_uneven_batch_config2_shape(dev):
    w = synth.workload(2, nq=24)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    offs = w.reads.offsets
    note(f"config-2 shape 24 reads M in [{w.reads.lengths.min()}, {w.reads.lengths.max()}]")
    check_i16(gpu_batch(dev, codes, qc, offs, sd.I16), qc, offs, codes)
    check_f32(gpu_batch(dev, z, qz, offs, sd.F32), qz, offs, z, index=np.arange(0, 24, 6))


def test_prepare_queries_matches_oracle(dev):
    w = synth.workload(2, nq=300)
    raw = torch.from_numpy(w.reads.values).to(dev)
    offs = torch.from_numpy(w.reads.offsets).to(dev)
    z, codes, nsat = sd.prepare_queries(raw, offs, 64.0)
    torch.cuda.synchronize()
    oz, oc, on = oracle.prepare_queries(w.reads.values, w.reads.offsets, 64.0)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), oz.view(np.uint32))
    assert np.array_equal(codes.cpu().numpy(), oc)
    assert int(nsat.item()) == on


@pytest.mark.parametrize("c", [0, 3])
def test_prepare_reference_matches_oracle(dev, c):
    # the joint statistics are accumulated in index order on the device, as
    # in the oracle's loop: z bits, codes and the saturation count are equal
    w = synth.workload(c, nq=1)
    g = torch.from_numpy(w.genome).to(dev)
    t = torch.from_numpy(w.table).to(dev)
    note(f"prepare_reference L={w.genome.size}")
    z, codes, nsat = sd.prepare_reference(g, t, 6, 64.0)
    torch.cuda.synchronize()
    oz, oc, on = oracle.prepare_reference(w.genome, w.table, 6, 64.0)
    assert np.array_equal(z.cpu().numpy().view(np.uint32), oz.view(np.uint32))
    assert np.array_equal(codes.cpu().numpy(), oc)
    assert int(nsat.item()) == on


@pytest.mark.parametrize("scale", [2.0, 32.0, 256.0])
def test_prepare_and_align_at_other_scales(dev, scale):
    # the fixed-point scale is a parameter (section 4.3 uses 2^5; section 6
    # sweeps it): device preparation of the reference and of the reads gives
    # the oracle's codes and saturation counts, and the int16 path on those
    # codes equals the exact integer oracle
    w = synth.workload(1, nq=256)
    g = torch.from_numpy(w.genome).to(dev)
    t = torch.from_numpy(w.table).to(dev)
    note(f"scale {scale}: preparation and 256 reads")
    _, codes, nsat = sd.prepare_reference(g, t, 6, scale)
    raw = torch.from_numpy(w.reads.values).to(dev)
    offs_dev = torch.from_numpy(w.reads.offsets).to(dev)
    _, qc, qnsat = sd.prepare_queries(raw, offs_dev, scale)
    torch.cuda.synchronize()
    _, oc, on = oracle.prepare_reference(w.genome, w.table, 6, scale)
    _, oqc, oqn = oracle.prepare_queries(w.reads.values, w.reads.offsets, scale)
    assert np.array_equal(codes.cpu().numpy(), oc) and int(nsat.item()) == on
    assert np.array_equal(qc.cpu().numpy(), oqc) and int(qnsat.item()) == oqn
    ref = sd.Reference(codes)
    plan = sd.Plan(w.reads.offsets, sd.I16)
    cost, end = sd.align_batch(ref, plan, qc)
    torch.cuda.synchronize()
    check_i16((cost.cpu().numpy(), end.cpu().numpy()), oqc, w.reads.offsets, oc)
    plan.close()
    ref.close()


def test_autotune_keeps_results_and_is_remembered(dev, small_ref):
    w, z, codes, qz, qc = small_ref
    offs = w.reads.offsets
    ref = sd.Reference(torch.from_numpy(codes).to(dev))
    plan = sd.Plan(offs, sd.I16)
    q = torch.from_numpy(qc).to(dev)
    note("autotune 64 x M=250 int16")
    cfg = sd.autotune(ref, plan, q, max_columns=4096)
    assert cfg["strip"] in (16, 32) and cfg["chains"] in (1, 2) and cfg["bands"] in (1, 2, 4)
    assert cfg["waves_per_cu"] % cfg["bands"] == 0
    assert cfg["band_rows"] == 0 or cfg["band_rows"] >= 65
    cost, end = sd.align_batch(ref, plan, q)
    torch.cuda.synchronize()
    check_i16((cost.cpu().numpy(), end.cpu().numpy()), qc, offs, codes)
    again = sd.Plan(offs, sd.I16)
    assert sd.use_tuned(ref, again) and again.config == cfg
    # another batch of the same shape class (66 reads of 240-260 rows: the
    # same quarter-octave buckets of count, median and longest) finds it
    rng = np.random.default_rng(5)
    lens = rng.integers(240, 261, size=66)
    similar = sd.Plan(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), sd.I16)
    assert sd.use_tuned(ref, similar) and similar.config == cfg
    other = sd.Plan(offs[:9], sd.I16)
    assert not sd.use_tuned(ref, other)
    for pl in (plan, again, similar, other):
        pl.close()
    ref.close()


def test_autotune_cache_file_is_read_by_a_new_process(tmp_path):
    # SDTW_TUNE_CACHE: one process tunes and writes the file, a fresh one
    # applies the shape without tuning
    import os
    import subprocess
    import textwrap
    path = tmp_path / "tune.txt"
    code = textwrap.dedent("""
        import sys, numpy as np, torch
        sys.path.insert(0, %r)
        import synth, oracle, paper_2211_07340_amd as sd
        w = synth.workload(1, nq=64)
        _, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
        _, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
        dev = torch.device("cuda:0")
        ref = sd.Reference(torch.from_numpy(codes).to(dev))
        plan = sd.Plan(w.reads.offsets, sd.I16)
        if sys.argv[1] == "tune":
            print(sd.autotune(ref, plan, torch.from_numpy(qc).to(dev), max_columns=4096))
        else:
            print(sd.use_tuned(ref, plan), plan.config)
        torch.cuda.synchronize()
    """) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SDTW_TUNE_CACHE=str(path))
    out1 = subprocess.run([sys.executable, "-c", code, "tune"], env=env, capture_output=True,
                          text=True, timeout=240)
    assert out1.returncode == 0, out1.stderr[-2000:]
    assert path.exists() and len(path.read_text().splitlines()) == 1
    out2 = subprocess.run([sys.executable, "-c", code, "use"], env=env, capture_output=True,
                          text=True, timeout=240)
    assert out2.returncode == 0, out2.stderr[-2000:]
    assert out2.stdout.strip().splitlines()[-1].startswith("True")
    assert out1.stdout.strip().splitlines()[-1] in out2.stdout
