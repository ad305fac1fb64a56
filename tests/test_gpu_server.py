"""Read Until server: every result it serves equals the oracle's on the read's
prefix (normalised with its first chunk), whatever the mix it ran in.

Two targets are served at once, as in the serving workload: the 29,903-base
genome and a 600,000-base one (1.2 M columns, past the 2^20 columns from
which streams switch to strip 32), so that chunks of both launch shapes
share the device.  A seeded sample of up to 32 served results per target is
checked against the oracle.  Under the mapping-quality rule the server also
serves the runner-up end of every resident row; a sample of those is checked
against the oracle's last row (fewer on the large target, whose rows cost
the oracle seconds each).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")


def _prefix_codes(raw, rows):
    mean, sdv = oracle.zstats(raw[:400])
    q, _ = oracle.quantize(oracle.zapply(raw[:rows], mean, sdv), 64.0)
    return q


@pytest.mark.parametrize("decision", ["cost", "mapq"])
def test_served_results_match_oracle(decision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    targets, codes_of, raws_of = [], [], []
    for i, L in enumerate((synth.SMALL_GENOME, 600_000)):
        genome = synth.make_genome(L, L)
        rd = synth.simulate_reads(genome, table, np.full(48, 2000), 0.5, 91 + i)
        raws = [rd.values[rd.offsets[r]:rd.offsets[r + 1]] for r in range(48)]
        # the reference codes come from the oracle, so that every input of the
        # check below is independent of the library
        _, codes, _ = oracle.prepare_reference(genome, table, 6)
        targets.append(srv.Target(f"{L}-base", sd.Reference(torch.from_numpy(codes).to(dev)),
                                  raws, np.asarray(rd.on_target, bool)))
        codes_of.append(codes)
        raws_of.append(raws)
    rec = []
    cfg = srv.ServerConfig(channels=32, decision=decision, mapq_window=700)
    server = srv.ReadUntilServer(targets, cfg, record=rec)
    server.calibrate(n_each=16)
    res = server.run(3.0, 0.5)
    print(decision, {k: res[k] for k in ("decisions", "decision_accuracy", "q_min", "tau")},
          flush=True)
    assert res["decisions"] > 20 and res["decision_accuracy"] > 0.9, res
    rng = np.random.default_rng(0)
    for t in range(2):
        mine = [r for r in rec if r[0] == t]
        assert mine, f"nothing served for target {t}"
        pick = [mine[i] for i in rng.choice(len(mine), min(32, len(mine)), replace=False)]
        qs = [_prefix_codes(raws_of[t][r[1]], r[2]) for r in pick]
        q, offs = synth.csr(qs)
        want_c, want_e, _ = oracle.batch(oracle.I64, q.astype(np.int16), offs, codes_of[t])
        got = [(r[3], r[4]) for r in pick]
        assert got == list(zip(want_c.astype(np.int64).tolist(), want_e.tolist())), t
        if decision != "mapq":
            assert all(r[5] is None for r in pick)
            continue
        for r, x in list(zip(pick, qs))[:8 if t == 0 else 2]:
            _, _, row = oracle.sdtw_i64(x, codes_of[t], lastrow=True)
            b, jb, s2, j2 = oracle.best_two(row, 700)
            assert (r[3], r[4]) == (int(b), jb)
            want = (np.iinfo(np.int32).max, -1) if j2 < 0 else (int(s2), j2)
            assert (r[5], r[6]) == want, (t, r)
    for t in targets:
        t.ref.close()


def test_raw_mode_served_results_match_oracle():
    # chunks of raw samples: events detected on the device from the samples
    # received so far; every served result equals the oracle's on the read's
    # first events (the oracle's events of the whole read: events written for
    # a prefix are final)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import events as oev
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    specs, codes_of, raws = [], [], []
    for i, L in enumerate((synth.SMALL_GENOME, 600_000)):
        genome = synth.make_genome(L, L)
        rr = synth.simulate_raw(genome, table, 24, 800, 0.5, 700 + i)
        specs.append((f"{L}-base", genome, table, rr.values, rr.offsets, rr.on_target))
        _, codes, _ = oracle.prepare_reference(genome, table, 6)
        codes_of.append(codes)
        raws.append(rr)
    targets = srv.make_raw_targets(specs, dev)
    cfg = srv.ServerConfig(channels=24, raw=True, max_events=1200, min_reject_events=800)
    rec = []
    server = srv.ReadUntilServer(targets, cfg, record=rec)
    server.calibrate(n_each=8)
    res = server.run(3.0, 0.5)
    print("raw mode", {k: res[k] for k in ("decisions", "decision_accuracy", "tau")}, flush=True)
    assert res["decisions"] > 10 and res["decision_accuracy"] > 0.9, res
    rng = np.random.default_rng(1)
    for t in range(2):
        mine = [r for r in rec if r[0] == t]
        assert mine, f"nothing served for target {t}"
        first_rows = {}
        for r in mine:
            first_rows[r[1]] = min(first_rows.get(r[1], 10 ** 9), r[2])
        pick = [mine[i] for i in rng.choice(len(mine), min(10, len(mine)), replace=False)]
        events = {}
        for _, pi, rows, cost, end, _, _ in pick:
            if pi not in events:
                rr = raws[t]
                events[pi] = oev.events(rr.values[rr.offsets[pi]:rr.offsets[pi + 1]])
            e = events[pi][50:50 + rows]
            assert e.size == rows
            assert first_rows[pi] == 400
            mean, sdv = oracle.zstats(e[:400])
            q, _ = oracle.quantize(oracle.zapply(e, mean, sdv), 64.0)
            assert (cost, end) == oracle.sdtw_i64(q, codes_of[t]), (t, pi, rows)
    for t in targets:
        t.ref.close()


def _check_records(rec, t, raws, codes, n, seed):
    """A seeded sample of n records of target t equals the int64 oracle on
    the read's prefix, normalised with its first chunk."""
    mine = [r for r in rec if r[0] == t]
    assert mine, f"nothing served for target {t}"
    rng = np.random.default_rng(seed)
    pick = [mine[i] for i in rng.choice(len(mine), min(n, len(mine)), replace=False)]
    qs = [_prefix_codes(raws[r[1]], r[2]) for r in pick]
    q, offs = synth.csr(qs)
    want_c, want_e, _ = oracle.batch(oracle.I64, q.astype(np.int16), offs, codes,
                                     nthreads=THREADS)
    got = [(r[3], r[4]) for r in pick]
    assert got == list(zip(want_c.astype(np.int64).tolist(), want_e.tolist())), t
    return len(pick), len(mine)


THREADS = 16


def _targets(dev, lengths, pool, seed):
    from paper_2211_07340_amd import server as srv
    table = synth.make_level_table()
    targets, codes_of, raws_of = [], [], []
    for i, L in enumerate(lengths):
        genome = synth.make_genome(L, L)
        rd = synth.simulate_reads(genome, table, np.full(pool, 2000), 0.5, seed + i)
        raws = [rd.values[rd.offsets[r]:rd.offsets[r + 1]] for r in range(pool)]
        _, codes, _ = oracle.prepare_reference(genome, table, 6)
        targets.append(srv.Target(f"{L}-base", sd.Reference(torch.from_numpy(codes).to(dev)),
                                  raws, np.asarray(rd.on_target, bool)))
        codes_of.append(codes)
        raws_of.append(raws)
    return targets, codes_of, raws_of


@pytest.mark.parametrize("wide", [-1, 0])
def test_large_target_served_results_match_oracle(wide):
    # the serving workload's two targets at their full sizes: the 29,903-base
    # genome and the 5,000,000-base genome (9,999,990 columns, 40 MB resident
    # rows); 32 served results of the large target and 16 of the small one
    # equal the oracle, with small batches extended over the whole device
    # (wide=-1, the calibrated default) and with batched launches only
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    targets, codes_of, raws_of = _targets(dev, (synth.SMALL_GENOME, synth.LARGE_GENOME), 32, 95)
    rec = []
    server = srv.ReadUntilServer(targets, srv.ServerConfig(channels=32, row_budget_bytes=8 << 30,
                                                           wide_chunks=wide),
                                 record=rec)
    cal = server.calibrate(n_each=8)
    res = server.run(4.0, 0.5)
    print("large target", wide, cal,
          {k: res[k] for k in ("decisions", "decision_accuracy", "wide_chunks", "per_target")},
          flush=True)
    assert res["decision_accuracy"] > 0.9, res
    assert (res["wide_chunks"] > 0) == (wide != 0), res
    n1, m1 = _check_records(rec, 1, raws_of[1], codes_of[1], 32, 5)
    n0, m0 = _check_records(rec, 0, raws_of[0], codes_of[0], 16, 6)
    print(f"checked {n1} of {m1} large-target and {n0} of {m0} small-target records",
          flush=True)
    assert n1 == 32
    for t in targets:
        t.ref.close()


def test_small_budget_admission_waits_keep_results():
    # a row budget of 8 rows of the 600,000-base target (4.8 MB each) for 32
    # channels: reads wait for admission and their chunks queue; what is
    # served still equals the oracle
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    targets, codes_of, raws_of = _targets(dev, (synth.SMALL_GENOME, 600_000), 32, 97)
    row_bytes = 4 * (((1_199_990 + 2047) // 2048) * 2048 + 2048)
    rec = []
    budget = 8 * row_bytes
    server = srv.ReadUntilServer(targets, srv.ServerConfig(channels=32, row_budget_bytes=budget),
                                 record=rec)
    server.calibrate(n_each=8, group=4)  # 4 rows at a time fit the budget
    res = server.run(3.0, 0.5)
    sd.set_row_budget(16 << 30)
    print("small budget", {k: res[k] for k in ("decisions", "admission_waits",
                                                "max_waiting_chunks")}, flush=True)
    assert res["admission_waits"] > 0 and res["decisions"] > 10, res
    for t in (0, 1):
        _check_records(rec, t, raws_of[t], codes_of[t], 16, 7 + t)
    for t in targets:
        t.ref.close()
