"""The paper's two sDTW-level experiments, on one MI355X (one JSON line each).

latency  Single-query sDTW latency against reference length (the paper's
         sDTW-only experiment, section 6): one on-target read of 250 events
         against the forward+reverse signal of seeded genomes from 10^3 to
         10^7 bases.  Reported per length: the one-wave synchronised kernel
         launched for the read alone (sdtw_align_one), the batched engine
         with the read as a one-read batch at its fastest launch shape
         (bands of rows over up to four waves), the whole-device row scan
         (sdtw_align_one_wide) at its automatic and at each tile width, and
         the paper's accelerator cycle model, N + 249 cycles at 100 MHz for
         250 processing elements (section 4.3), as context.
scale    Accuracy against the fixed-point scaling factor (section 6): for
         scales 2, 4, ..., 256, the percentage of reads whose end position on
         the int16 path equals the float32 path's, and the number of values
         that saturate int16, on the 4,096-read workload (50% on-target).

serving  The Read Until server (workload 4) against the channel count and the
         row budget: reads/s, decision latency per target, admission waits,
         for the 29,903-base target alone and for both targets (50/50), and
         with a budget that holds only part of the large target's rows.
decision The two decision rules of the server (per-event cost threshold and
         the mapping-quality score from best and runner-up ends, section 5.1)
         on both targets at 512 channels, with off-target reads that are
         i.i.d. noise and, harder, pore signal of a 1,000,000-base background
         genome, every read at one noise level and (--noise-spread) each read
         at its own, 1x to 4x: accuracy, on-target reads kept, off-target
         reads rejected, mean events read before the decision, reads/s and
         latency.
events   Pre-processing on the device (section 4.1's event detection, prefix
         trimming and normalisation) against alignment, for 4,096 simulated
         raw reads (30 adaptor levels, then 320 bases; 50% on-target) and the
         29,903-base genome: device time per stage (HIP events, median of
         --reps), raw samples per second, and the share of each stage (the
         paper's pre-processing takes about 30% of its run time, section 6).
serving_raw  The Read Until server on raw samples (events detected on the
         device from the samples received so far, every batch), both
         targets, 512 channels, 2,400 samples per channel per 0.1 s chunk
         period, reads of 30 adaptor levels and 1,400 bases: reads/s,
         accuracy, decision latency per target; beside the same server on
         pre-detected events.
wide     The whole-device single-query scan alone (sdtw_align_one_wide) on
         one genome length (--genome, default 5,000,000 bases) at one width
         (--cols, default automatic): device time per call, median of
         --reps calls (HIP events), for a kernel trace of exactly that case.
issue    VALU issue rates on gfx950 (libsdtw_probe.so): cycles per 64-lane
         wave instruction per SIMD for v_min3_u32, v_sad_u32, v_sub_f32,
         v_add_f32 |a| and v_add_u32, by independent chains per wave (1, 2,
         4) and waves per SIMD (1-8), at the nominal 2.4 GHz clock: the basis
         of the cycles per cell of the roof in bench.py.
placement Where the hardware places the batch alignment's workgroups and
         waves (XCC, shader engine, CU, SIMD) against the order in which
         they take their first read.
lds      LDS cost of the tile switch's operations (libsdtw_probe.so): blocks
         of 8 ds_read_b128 + 8 ds_write_b128 per wave with 1, 16 or 64 lanes
         active, cycles per LDS instruction per CU by waves per SIMD.
best_two The runner-up search alone (sdtw_stream_best_two) over 1 to 256
         resident rows of the 5,000,000-base target (9,999,990 columns):
         device time and the rate at which it reads the rows (4 bytes per
         column per row, the bound being HBM at 8 TB/s).
stream_wide Extending 1 to 64 streams by one 400-event chunk each against
         the 5,000,000-base target: one batched launch against one
         whole-device call per chunk (sdtw_stream_extend_wide).
stream_batch The batched stream extension alone: --stream-chunks resident
         rows (default 256) extended by a 400-event chunk each against the
         5,000,000-base target, by launch shape (--stream-shapes, strip:bands,
         0:0 for the library's choice): one batch alone (HIP events) and two
         such batches issued at once on two HIP streams (host clock around
         both), as the server keeps two batches per target in flight; the
         fraction of the VALU roof of each.

Usage: python bench_experiments.py latency|scale|serving|serving_raw|decision|best_two|wide|events|issue|lds|placement|stream_wide|stream_batch
                                   [--max-genome BASES] [--genome BASES] [--cols C]
                                   [--reps R]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (sets the hardware queue count before HIP starts)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_ms(torch, fn, reps: int) -> float:
    """Median device time of fn() over reps launches (HIP events on the
    current stream), after one warm-up."""
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = _events(torch)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def latency(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    lengths = [1_000, 10_000, 29_903, 128_920, 1_000_000, 5_000_000, 10_000_000]
    lengths = [L for L in lengths if L <= args.max_genome]
    for L in lengths:
        genome = synth.make_genome(L, L)
        rd = synth.simulate_reads(genome, table, [250], 1.0, 7000 + L % 997)
        g = torch.from_numpy(genome).to(dev)
        tab = torch.from_numpy(table).to(dev)
        _, cref, _ = sd.prepare_reference(g, tab, 6, 64.0)
        ref = sd.Reference(cref)
        raw = torch.from_numpy(rd.values).to(dev)
        offs = torch.from_numpy(rd.offsets).to(dev)
        _, q, _ = sd.prepare_queries(raw, offs, 64.0)
        N = ref.n
        reps = 20 if N < 3_000_000 else 5
        one = _time_ms(torch, lambda: sd.align_one(ref, q), reps)
        plan = sd.Plan(rd.offsets, sd.I16)
        best = None
        for strip, bands in ((16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4)):
            plan.set_config(strip=strip, chains=1, bands=bands, waves_per_cu=4 * bands)
            ms = _time_ms(torch, lambda: sd.align_batch(ref, plan, q), reps)
            if best is None or ms < best[0]:
                best = (ms, strip, bands)
        wide = {}
        for cols in (8, 16, 32, 64, 0):
            wide[cols] = _time_ms(torch, lambda: sd.align_one_wide(ref, q, cols=cols), reps)
        c1, e1 = sd.align_one(ref, q)
        plan.set_config(strip=best[1], chains=1, bands=best[2], waves_per_cu=4 * best[2])
        c2, e2 = sd.align_batch(ref, plan, q)
        c3, e3 = sd.align_one_wide(ref, q)
        torch.cuda.synchronize()
        assert (int(c1.item()), int(e1.item())) == (int(c2.item()), int(e2.item()))
        assert (int(c1.item()), int(e1.item())) == (int(c3.item()), int(e3.item()))
        wbest = min((v, k) for k, v in wide.items() if k)
        cells = 250.0 * N
        fpga_ms = (N + 249) / 100e6 * 1e3
        print(json.dumps({
            "experiment": "sdtw latency vs reference length", "genome_bases": L,
            "reference_values": N, "query_events": 250,
            "one_wave_ms": round(one, 4), "one_wave_gcups": round(cells / one / 1e6, 2),
            "banded_ms": round(best[0], 4), "banded_gcups": round(cells / best[0] / 1e6, 2),
            "banded_shape": {"strip": best[1], "bands": best[2]},
            "row_scan_ms": round(wide[0], 4), "row_scan_gcups": round(cells / wide[0] / 1e6, 2),
            "row_scan_best_ms": round(wbest[0], 4), "row_scan_best_cols": wbest[1],
            "row_scan_ms_by_cols": {str(k): round(v, 4) for k, v in wide.items() if k},
            "paper_accelerator_model_ms": round(fpga_ms, 4),
            "end": int(e1.item())}), flush=True)
        plan.close()
        ref.close()


def scale(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    w = synth.workload(1)
    reads = w.reads
    g = torch.from_numpy(w.genome).to(dev)
    tab = torch.from_numpy(w.table).to(dev)
    raw = torch.from_numpy(reads.values).to(dev)
    offs = torch.from_numpy(reads.offsets).to(dev)
    zref, _, _ = sd.prepare_reference(g, tab, w.k, 64.0)
    fref = sd.Reference(zref)
    zq, _, _ = sd.prepare_queries(raw, offs, 64.0)
    fplan = sd.Plan(reads.offsets, sd.F32)
    _, fend = sd.align_batch(fref, fplan, zq)
    torch.cuda.synchronize()
    fend = fend.cpu().numpy()
    on = reads.on_target
    for s in (2, 4, 8, 16, 32, 64, 128, 256):
        _, cref, rsat = sd.prepare_reference(g, tab, w.k, float(s))
        _, cq, qsat = sd.prepare_queries(raw, offs, float(s))
        iref = sd.Reference(cref)
        iplan = sd.Plan(reads.offsets, sd.I16)
        _, iend = sd.align_batch(iref, iplan, cq)
        torch.cuda.synchronize()
        iend = iend.cpu().numpy()
        same = iend == fend
        print(json.dumps({
            "experiment": "end position vs fixed-point scale", "scale": s,
            "reads": int(reads.nq),
            "pct_end_equal_all": round(100 * float(same.mean()), 2),
            "pct_end_equal_on_target": round(100 * float(same[on].mean()), 2),
            "pct_end_within_10_on_target": round(
                100 * float((np.abs(iend - fend) <= 10)[on].mean()), 2),
            "saturated_reference_values": int(rsat), "saturated_query_values": int(qsat)}),
            flush=True)
        iplan.close()
        iref.close()
    fplan.close()
    fref.close()


def serving(args):
    import torch

    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    small = bench.serving_targets(torch, dev, large=False)
    both = bench.serving_targets(torch, dev, large=True)
    chans = lambda v: [int(x) for x in v.split(",") if x]  # noqa: E731
    wides = [int(x) for x in args.wide_chunks.split(",")]
    runs = [("29,903-base only", small, ch, 64 << 30, w) for ch in chans(args.small_channels)
            for w in wides]
    runs += [("both targets", both, ch, 64 << 30, w) for ch in chans(args.both_channels)
             for w in wides]
    if args.budget_run:
        runs += [("both targets", both, 256, 4 << 30, wides[0])]  # about 100 large rows
    for name, targets, ch, budget, wide in runs:
        cfg = srv.ServerConfig(channels=ch, row_budget_bytes=budget, wide_chunks=wide)
        server = srv.ReadUntilServer(targets, cfg, mode="extend")
        cal = server.calibrate()
        r = server.run(8.0, 3.0)
        print(json.dumps({"experiment": "serving", "targets": name, "channels": ch,
                          "row_budget_gib": budget >> 30, "wide_chunks_setting": wide,
                          "wide_max": {k: v["wide_max"] for k, v in cal.items()},
                          **{k: r[k] for k in ("reads_per_s", "chunks_per_s", "gcups",
                                               "decision_latency_p50_ms",
                                               "decision_latency_p99_ms", "admission_waits",
                                               "max_waiting_chunks", "decision_accuracy",
                                               "wide_chunks")},
                          "per_target": r["per_target"]}), flush=True)
    for t in small + both:
        t.ref.close()


def stream_wide(args):
    """Extending k streams by one 400-event chunk each against the
    9,999,990-column reference: one batched launch (sdtw_stream_extend)
    against k whole-device calls (sdtw_stream_extend_wide); HIP events, best
    of two, after each stream's first chunk."""
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    w = synth.workload(3, nq=1)
    g = torch.from_numpy(w.genome).to(dev)
    t = torch.from_numpy(w.table).to(dev)
    _, cref, _ = sd.prepare_reference(g, t, 6, 64.0)
    ref = sd.Reference(cref)
    sd.set_row_budget(64 << 30)
    rng = np.random.default_rng(5)
    M = 400
    for k in [int(v) for v in args.chunks.split(",")]:
        streams = [sd.Stream(ref) for _ in range(k)]
        offs = np.arange(k + 1, dtype=np.int64) * M
        q = torch.from_numpy(rng.integers(-300, 300, size=k * M).astype(np.int16)).to(dev)
        sd.stream_extend(streams, q, offs)  # first chunk
        torch.cuda.synchronize()
        res = {"batch": [], "wide": []}
        for way in ("batch", "wide") * 2:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            if way == "batch":
                sd.stream_extend(streams, q, offs)
            else:
                for i in range(k):
                    sd.stream_extend_wide(streams[i], q[i * M:(i + 1) * M])
            b.record()
            b.synchronize()
            res[way].append(a.elapsed_time(b))
        bm, wm = min(res["batch"]), min(res["wide"])
        print(json.dumps({"experiment": "stream extension, batched against whole device",
                          "chunks": k, "rows": M, "reference_values": ref.n,
                          "batch_ms": round(bm, 2), "wide_ms": round(wm, 2),
                          "wide_ms_per_chunk": round(wm / k, 3)}), flush=True)
        torch.cuda.synchronize()
        for s_ in streams:
            s_.close()
    ref.close()


def stream_batch(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    w = synth.workload(3, nq=1)
    g = torch.from_numpy(w.genome).to(dev)
    t = torch.from_numpy(w.table).to(dev)
    _, cref, _ = sd.prepare_reference(g, t, 6, 64.0)
    ref = sd.Reference(cref)
    sd.set_row_budget(64 << 30)
    rng = np.random.default_rng(5)
    M, k = 400, args.stream_chunks
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    roof = bench.valu_peak_tcups("i16")
    for shape in args.stream_shapes.split(","):
        strip, bands = (int(v) for v in shape.split(":"))
        sd.set_stream_config(strip, bands, ref=ref)
        streams = [sd.Stream(ref) for _ in range(2 * k)]
        offs = np.arange(k + 1, dtype=np.int64) * M
        q = torch.from_numpy(rng.integers(-300, 300, size=k * M).astype(np.int16)).to(dev)
        with torch.cuda.stream(hs[0]):
            sd.stream_extend(streams[:k], q, offs, stream=hs[0])  # first chunk of each row
            sd.stream_extend(streams[k:], q, offs, stream=hs[0])
        torch.cuda.synchronize()
        one, two = [], []
        # each rep extends the first k rows twice: stay within 4,096 rows
        for _ in range(max(1, min(args.reps, (4096 // M - 1) // 2))):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(hs[0])
            sd.stream_extend(streams[:k], q, offs, stream=hs[0])
            b.record(hs[0])
            b.synchronize()
            one.append(a.elapsed_time(b))
            if not args.stream_two:
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sd.stream_extend(streams[:k], q, offs, stream=hs[0])
            sd.stream_extend(streams[k:], q, offs, stream=hs[1])
            torch.cuda.synchronize()
            two.append((time.perf_counter() - t0) * 1e3)
        cells = k * M * ref.n
        o = min(one)
        rec = {"experiment": "stream_batch", "chunks": k, "rows": M,
               "reference_values": ref.n, "strip": strip, "bands": bands,
               "one_batch_ms": round(o, 2), "frac_one": round(cells / o / 1e9 / roof, 3)}
        if two:
            rec.update(two_batches_ms=round(min(two), 2),
                       frac_two=round(2 * cells / min(two) / 1e9 / roof, 3))
        print(json.dumps(rec), flush=True)
        for s_ in streams:
            s_.close()
    sd.set_stream_config(0, 0, ref=ref)
    ref.close()


def decision(args):
    import torch

    import synth
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    background = synth.make_genome(1_000_000, 1_000_003)
    for off, spread in ((o, float(sp)) for sp in args.noise_spread.split(",")
                        for o in args.off.split(",")):
        specs = []
        for i, (name, L) in enumerate((("29,903-base", synth.SMALL_GENOME),
                                       ("5,000,000-base", synth.LARGE_GENOME))):
            genome = synth.make_genome(L, L)
            rd = synth.simulate_reads(genome, table, np.full(512, 2000), 0.5, 4400 + i,
                                      off_genome=background if off == "genomic" else None,
                                      noise_spread=spread)
            raws = [rd.values[rd.offsets[r]:rd.offsets[r + 1]] for r in range(512)]
            specs.append((name, genome, table, raws, rd.on_target))
        targets = srv.make_targets(specs, dev)
        for rule in ("cost", "mapq"):
            cfg = srv.ServerConfig(channels=512, row_budget_bytes=64 << 30, decision=rule)
            server = srv.ReadUntilServer(targets, cfg, mode="extend")
            server.calibrate()
            r = server.run(8.0, 3.0)
            print(json.dumps({"experiment": "decision rule", "off_target_reads": off,
                              "noise_spread": spread, "rule": rule,
                              **{k: r[k] for k in ("reads_per_s", "decision_accuracy",
                                                   "on_target_kept", "off_target_rejected",
                                                   "mean_events_at_decision", "tau", "q_min",
                                                   "decision_latency_p50_ms",
                                                   "decision_latency_p99_ms")},
                              "per_target": r["per_target"]}), flush=True)
        for t in targets:
            t.ref.close()


def serving_raw(args):
    import torch

    import synth
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    specs = []
    for i, (name, L) in enumerate((("29,903-base", synth.SMALL_GENOME),
                                   ("5,000,000-base", synth.LARGE_GENOME))):
        genome = synth.make_genome(L, L)
        rr = synth.simulate_raw(genome, table, 512, 1400, 0.5, 4600 + i)
        specs.append((name, genome, table, rr.values, rr.offsets, rr.on_target))
    targets = srv.make_raw_targets(specs, dev)
    for ch in (128, 512):
        cfg = srv.ServerConfig(channels=ch, row_budget_bytes=64 << 30, raw=True)
        server = srv.ReadUntilServer(targets, cfg, mode="extend")
        server.calibrate()
        r = server.run(8.0, 3.0)
        print(json.dumps({"experiment": "serving from raw samples", "channels": ch,
                          "chunk_samples": cfg.chunk_samples,
                          **{k: r[k] for k in ("reads_per_s", "chunks_per_s", "gcups",
                                               "decision_accuracy", "mean_events_at_decision",
                                               "decision_latency_p50_ms",
                                               "decision_latency_p99_ms")},
                          "per_target": r["per_target"],
                          "host_loop_ms": r["host_loop_ms"]}), flush=True)
    for t in targets:
        t.ref.close()


def events(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    genome = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    raw = synth.simulate_raw(genome, table, 4096, 320, 0.5, 4242)
    x = torch.from_numpy(raw.values).to(dev)
    xo = torch.from_numpy(raw.offsets).to(dev)
    _, cref, _ = sd.prepare_reference(torch.from_numpy(genome).to(dev),
                                      torch.from_numpy(table).to(dev), synth.K, 64.0)
    ref = sd.Reference(cref)
    ev, cnt = sd.detect_events(x, xo, 50, 250)
    torch.cuda.synchronize()
    assert bool((cnt == 250).all())
    eo_np = np.arange(4097, dtype=np.int64) * 250
    eo = torch.from_numpy(eo_np).to(dev)
    _, q, _ = sd.prepare_queries(ev.reshape(-1), eo, 64.0)
    plan = sd.Plan(eo_np, sd.I16)
    sd.autotune(ref, plan, q)
    reps = args.reps
    t_ev = _time_ms(torch, lambda: sd.detect_events(x, xo, 50, 250), reps)
    t_norm = _time_ms(torch, lambda: sd.prepare_queries(ev.reshape(-1), eo, 64.0), reps)
    t_al = _time_ms(torch, lambda: sd.align_batch(ref, plan, q), reps)
    total = t_ev + t_norm + t_al
    print(json.dumps({"experiment": "pre-processing vs alignment", "reads": 4096,
                      "raw_samples": int(raw.values.size),
                      "events_per_read": 250, "trim": 50,
                      "detect_events_ms": round(t_ev, 4), "normalise_ms": round(t_norm, 4),
                      "align_ms": round(t_al, 4),
                      "raw_samples_per_s": round(raw.values.size / (t_ev * 1e-3), 1),
                      "reads_per_s_end_to_end": round(4096 / (total * 1e-3), 1),
                      "share_detect_events": round(t_ev / total, 4),
                      "share_normalise": round(t_norm / total, 4),
                      "share_align": round(t_al / total, 4)}), flush=True)
    plan.close()
    ref.close()


def wide(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    L = args.genome
    genome = synth.make_genome(L, L)
    rd = synth.simulate_reads(genome, table, [250], 1.0, 7000 + L % 997)
    _, cref, _ = sd.prepare_reference(torch.from_numpy(genome).to(dev),
                                      torch.from_numpy(table).to(dev), synth.K, 64.0)
    ref = sd.Reference(cref)
    _, q, _ = sd.prepare_queries(torch.from_numpy(rd.values).to(dev),
                                 torch.from_numpy(rd.offsets).to(dev), 64.0)
    ms = _time_ms(torch, lambda: sd.align_one_wide(ref, q, cols=args.cols), args.reps)
    c, e = sd.align_one_wide(ref, q, cols=args.cols)
    torch.cuda.synchronize()
    print(json.dumps({"experiment": "wide", "genome_bases": L, "reference_values": ref.n,
                      "query_events": 250, "cols": args.cols, "reps": args.reps,
                      "ms_median": round(ms, 4), "gcups": round(250.0 * ref.n / ms / 1e6, 1),
                      "cost": int(c.item()), "end": int(e.item())}), flush=True)
    ref.close()


def best_two(args):
    import torch

    import synth
    import paper_2211_07340_amd as sd
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    genome = synth.make_genome(synth.LARGE_GENOME, synth.LARGE_GENOME)
    _, cref, _ = sd.prepare_reference(torch.from_numpy(genome).to(dev),
                                      torch.from_numpy(table).to(dev), synth.K, 64.0)
    ref = sd.Reference(cref)
    rd = synth.simulate_reads(genome, table, np.full(256, 400), 0.5, 515)
    _, q, _ = sd.prepare_queries(torch.from_numpy(rd.values).to(dev),
                                 torch.from_numpy(rd.offsets).to(dev), 64.0)
    streams = [sd.Stream(ref) for _ in range(256)]
    sd.stream_extend(streams, q, rd.offsets)
    torch.cuda.synchronize()
    for ns in (1, 8, 64, 256):
        ms = _time_ms(torch, lambda: sd.stream_best_two(streams[:ns], 2000), 10)
        gbs = ns * 4.0 * ref.n / (ms * 1e-3) / 1e9
        print(json.dumps({"experiment": "best_two", "rows": ns, "columns": ref.n,
                          "ms": round(ms, 4), "row_read_gb_per_s": round(gbs, 1),
                          "hbm_fraction": round(gbs / 8000.0, 3)}), flush=True)
    for st in streams:
        st.close()
    ref.close()


def issue(args):
    """VALU issue rates (libsdtw_probe.so): cycles per 64-lane wave instruction
    per SIMD for the instruction kinds of the cell update, by independent
    chains per wave and waves per SIMD; the basis of the roof in bench.py."""
    import ctypes as C

    import torch
    from paper_2211_07340_amd import build as hipbuild
    lib = C.CDLL(hipbuild.PROBE_LIB)
    lib.sdtw_probe_issue.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                     C.c_void_p]
    lib.sdtw_probe_issue.restype = C.c_int
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    clock_ghz = 2.4  # nominal engine clock of the MI355X
    out = torch.empty(4 * cus * 8 * 64, dtype=torch.int32, device="cuda")
    kinds = ["v_min3_u32", "v_sad_u32", "v_sub_f32", "v_add_f32 |a|", "v_add_u32"]
    st = torch.cuda.current_stream()
    for k, name in enumerate(kinds):
        for chains in (1, 2, 4):
            for waves in (1, 2, 3, 4, 8):
                # 640,000 instructions per SIMD (about a millisecond): the
                # launch itself is noise
                iters = 40000 // (waves * chains)

                def run():
                    rc = lib.sdtw_probe_issue(k, chains, waves, iters, C.c_void_p(out.data_ptr()),
                                              C.c_void_p(st.cuda_stream))
                    assert rc == 0, rc
                ms = _time_ms(torch, run, 3)
                instr_per_simd = waves * iters * 16 * chains
                cyc = ms * 1e-3 * clock_ghz * 1e9 / instr_per_simd
                print(json.dumps({"experiment": "issue", "instruction": name, "chains": chains,
                                  "waves_per_simd": waves, "ms": round(ms, 3),
                                  "cycles_per_wave_instr_per_simd": round(cyc, 2),
                                  "cycles_per_wave_instr_per_wave": round(cyc * waves, 2)}),
                      flush=True)


def lds(args):
    """LDS cost of the tile switch's operations (libsdtw_probe.so): blocks of
    8 ds_read_b128 + 8 ds_write_b128 per wave with 1 or 64 lanes active;
    cycles per LDS instruction per CU by waves per SIMD."""
    import ctypes as C

    import torch
    from paper_2211_07340_amd import build as hipbuild
    lib = C.CDLL(hipbuild.PROBE_LIB)
    lib.sdtw_probe_lds.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    lib.sdtw_probe_lds.restype = C.c_int
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    clock_ghz = 2.4
    out = torch.empty(4 * cus * 8 * 64, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    for lanes in (1, 16, 64):
        for waves in (1, 2, 4, 8):
            iters = 8000 // waves

            def run():
                rc = lib.sdtw_probe_lds(lanes, waves, iters, C.c_void_p(out.data_ptr()),
                                        C.c_void_p(st.cuda_stream))
                assert rc == 0, rc
            ms = _time_ms(torch, run, 3)
            per_cu = 4 * waves * iters * 16
            print(json.dumps({"experiment": "lds", "lanes": lanes, "waves_per_simd": waves,
                              "ms": round(ms, 3),
                              "cycles_per_lds_instr_per_cu": round(
                                  ms * 1e-3 * clock_ghz * 1e9 / per_cu, 2),
                              "cycles_per_block_per_wave": round(
                                  ms * 1e-3 * clock_ghz * 1e9 / iters, 1)}), flush=True)


def placement(args):
    """Where the hardware places the batch alignment's workgroups
    (libsdtw_probe.so): the 2-band launch of workload 3 (1,024 workgroups of
    128 threads, 230 vector registers per wave and the same dynamic LDS) and
    the 1-band one (1,024 of 64 threads, 150 registers, the LDS share that
    spreads four over every compute unit), each workgroup's first ticket (the
    persistent kernel's first read), the XCC, shader engine, CU and SIMD of
    each of its waves, and whether every wave was resident at once."""
    import collections
    import ctypes as C

    import torch
    from paper_2211_07340_amd import build as hipbuild
    lib = C.CDLL(hipbuild.PROBE_LIB)
    lib.sdtw_probe_placement.argtypes = [C.c_int] * 5 + [C.c_void_p] * 2
    lib.sdtw_probe_placement.restype = C.c_int
    st = torch.cuda.current_stream()
    for blocks, threads, lds, vgprs in ((1024, 128, 37968, 230), (1024, 64, 39936, 150)):
        wpb = threads // 64
        o32 = torch.zeros(8 + 8 * blocks * wpb, dtype=torch.int32, device="cuda")
        rc = lib.sdtw_probe_placement(blocks, threads, lds, vgprs, 2000,
                                      C.c_void_p(o32.data_ptr()), C.c_void_p(st.cuda_stream))
        assert rc == 0, rc
        torch.cuda.synchronize()
        rec = o32[8:].view(blocks, wpb, 8).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        cus, simds = collections.Counter(), collections.Counter()
        rows = []
        for b in range(blocks):
            locs = []
            for wv in range(wpb):
                hw, xcc = int(rec[b, wv, 1]), int(rec[b, wv, 2])
                cu = (xcc & 0xF, (hw >> 13) & 7, (hw >> 12) & 1, (hw >> 8) & 15)
                simd = cu + ((hw >> 4) & 3,)
                cus[cu] += 1
                simds[simd] += 1
                locs.append(list(simd))
            rows.append({"block": b, "ticket": int(rec[b, 0, 0]), "waves": locs,
                         "t0": int(rec[b, 0, 3]), "t1": int(rec[b, 0, 4])})
        t0 = rec[:, :, 3].astype(np.int64)
        t1 = rec[:, :, 4].astype(np.int64)
        print(json.dumps({"experiment": "placement", "blocks": blocks, "threads": threads,
                          "lds_bytes": lds, "vgprs": vgprs, "cus_used": len(cus),
                          "waves_per_cu": sorted(collections.Counter(cus.values()).items()),
                          "simds_used": len(simds),
                          "waves_per_simd": sorted(collections.Counter(simds.values()).items()),
                          "same_simd_workgroups": sum(
                              1 for r in rows if len({tuple(w) for w in r["waves"]}) < wpb),
                          "all_resident_together": bool(t0.max() < t1.min()),
                          "start_spread_us": float(t0.max() - t0.min()) / 100.0,
                          "first_blocks": rows[:8]}), flush=True)
        with open(os.path.join(args.out_dir, f"placement_{threads}.json"), "w") as f:
            json.dump(rows, f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment",
                    choices=["latency", "scale", "serving", "serving_raw", "decision",
                             "best_two", "wide", "events", "issue", "lds", "placement",
                             "stream_wide", "stream_batch"])
    ap.add_argument("--max-genome", type=int, default=10_000_000)
    ap.add_argument("--genome", type=int, default=5_000_000, help="wide: genome bases")
    ap.add_argument("--cols", type=int, default=0, help="wide: columns per thread (0: auto)")
    ap.add_argument("--reps", type=int, default=20, help="wide: timed calls")
    ap.add_argument("--out-dir", default=".", help="placement: where the records go")
    ap.add_argument("--off", default="noise,genomic",
                    help="decision: off-target read kinds to run, in order")
    ap.add_argument("--chunks", default="1,4,16,64",
                    help="stream_wide: numbers of streams extended per call")
    ap.add_argument("--stream-chunks", type=int, default=256,
                    help="stream_batch: resident rows extended per batch")
    ap.add_argument("--stream-shapes", default="0:0,32:4,32:2,16:4",
                    help="stream_batch: launch shapes strip:bands (0:0: the library's)")
    ap.add_argument("--stream-two", type=int, default=1,
                    help="stream_batch: also time two batches issued at once (0: one only)")
    ap.add_argument("--small-channels", default="512,1024,2048",
                    help="serving: channel counts with the 29,903-base target alone")
    ap.add_argument("--both-channels", default="64,128,256,512",
                    help="serving: channel counts with both targets")
    ap.add_argument("--wide-chunks", default="-1",
                    help="serving: ServerConfig.wide_chunks settings to run (-1: calibrated, "
                         "0: batched launches only)")
    ap.add_argument("--budget-run", type=int, default=1,
                    help="serving: also run 256 channels with a 4 GiB row budget")
    ap.add_argument("--noise-spread", default="1,4",
                    help="decision: per-read noise spreads to run (1: every read at the "
                         "same noise level; s: each read's noise 1x to s x, log-uniform)")
    args = ap.parse_args()
    t0 = time.perf_counter()
    {"latency": latency, "scale": scale, "serving": serving,
     "decision": decision, "best_two": best_two, "wide": wide,
     "events": events, "serving_raw": serving_raw, "issue": issue,
     "lds": lds, "placement": placement, "stream_wide": stream_wide,
     "stream_batch": stream_batch}[args.experiment](args)
    print(json.dumps({"done": args.experiment, "seconds": round(time.perf_counter() - t0, 1)}),
          flush=True)


if __name__ == "__main__":
    main()
