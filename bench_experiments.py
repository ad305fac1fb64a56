"""The paper's two sDTW-level experiments, on one MI355X (one JSON line each).

latency  Single-query sDTW latency against reference length (the paper's
         sDTW-only experiment, section 6): one on-target read of 250 events
         against the forward+reverse signal of seeded genomes from 10^3 to
         10^7 bases.  Reported per length: the one-wave synchronised kernel
         launched for the read alone (sdtw_align_one), the batched engine
         with the read as a one-read batch at its fastest launch shape
         (bands of rows over up to four waves), and the paper's accelerator
         cycle model, N + 249 cycles at 100 MHz for 250 processing elements
         (section 4.3), as context.
scale    Accuracy against the fixed-point scaling factor (section 6): for
         scales 2, 4, ..., 256, the percentage of reads whose end position on
         the int16 path equals the float32 path's, and the number of values
         that saturate int16, on the 4,096-read workload (50% on-target).

serving  The Read Until server (workload 4) against the channel count and the
         row budget: reads/s, decision latency per target, admission waits,
         for the 29,903-base target alone and for both targets (50/50), and
         with a budget that holds only part of the large target's rows.

Usage: python bench_experiments.py latency|scale|serving [--max-genome BASES]
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
        c1, e1 = sd.align_one(ref, q)
        plan.set_config(strip=best[1], chains=1, bands=best[2], waves_per_cu=4 * best[2])
        c2, e2 = sd.align_batch(ref, plan, q)
        torch.cuda.synchronize()
        assert (int(c1.item()), int(e1.item())) == (int(c2.item()), int(e2.item()))
        cells = 250.0 * N
        fpga_ms = (N + 249) / 100e6 * 1e3
        print(json.dumps({
            "experiment": "sdtw latency vs reference length", "genome_bases": L,
            "reference_values": N, "query_events": 250,
            "one_wave_ms": round(one, 4), "one_wave_gcups": round(cells / one / 1e6, 2),
            "banded_ms": round(best[0], 4), "banded_gcups": round(cells / best[0] / 1e6, 2),
            "banded_shape": {"strip": best[1], "bands": best[2]},
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
    runs = [("29,903-base only", small, ch, 64 << 30) for ch in (512, 1024, 2048)]
    runs += [("both targets", both, ch, 64 << 30) for ch in (64, 128, 256, 512)]
    runs += [("both targets", both, 256, 4 << 30)]  # about 100 large-target rows
    for name, targets, ch, budget in runs:
        cfg = srv.ServerConfig(channels=ch, row_budget_bytes=budget)
        server = srv.ReadUntilServer(targets, cfg, mode="extend")
        server.calibrate()
        r = server.run(8.0, 3.0)
        print(json.dumps({"experiment": "serving", "targets": name, "channels": ch,
                          "row_budget_gib": budget >> 30,
                          **{k: r[k] for k in ("reads_per_s", "chunks_per_s", "gcups",
                                               "decision_latency_p50_ms",
                                               "decision_latency_p99_ms", "admission_waits",
                                               "max_waiting_chunks", "decision_accuracy")},
                          "per_target": r["per_target"]}), flush=True)
    for t in small + both:
        t.ref.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["latency", "scale", "serving"])
    ap.add_argument("--max-genome", type=int, default=10_000_000)
    args = ap.parse_args()
    t0 = time.perf_counter()
    {"latency": latency, "scale": scale, "serving": serving}[args.experiment](args)
    print(json.dumps({"done": args.experiment, "seconds": round(time.perf_counter() - t0, 1)}),
          flush=True)


if __name__ == "__main__":
    main()
