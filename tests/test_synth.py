"""Seeded workload generator: shapes, determinism, and that on-target reads
really come from the reference (checked with the oracle)."""
import numpy as np

import oracle
import synth


def test_shapes_and_determinism():
    w = synth.workload(1)
    assert w.reads.nq == 4096 and np.all(w.reads.lengths == 250)
    assert w.genome.size == 29_903 and w.table.size == 4096
    w2 = synth.workload(1)
    assert np.array_equal(w.reads.values, w2.reads.values)
    assert 0.45 < w.reads.on_target.mean() < 0.55
    w2 = synth.workload(2)
    L = w2.reads.lengths
    assert w2.reads.nq == 8192 and L.min() >= 100 and L.max() <= 2000
    assert 0.65 < w2.reads.on_target.mean() < 0.75
    sub = synth.workload(1, nq=10)
    assert np.array_equal(sub.reads.values, w.reads.values[:2500])


def test_reference_size_is_two_strands_of_kmers():
    w = synth.workload(0)
    z, codes, nsat = oracle.prepare_reference(w.genome, w.table, w.k)
    assert z.size == 2 * (29_903 - 6 + 1) == 59_796
    assert abs(float(z.astype(np.float64).mean())) < 1e-6
    assert nsat == 0 and codes.dtype == np.int16


def test_on_target_reads_map_to_their_origin():
    w = synth.workload(1, nq=24)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    cost, end, _ = oracle.batch(oracle.F32, qz, w.reads.offsets, z)
    on = w.reads.on_target
    assert on.any() and (~on).any()
    assert np.all(np.abs(end[on] - w.reads.end_true[on]) <= 10)
    # on-target reads align far more cheaply than off-target ones
    assert cost[on].max() < cost[~on].min()
    ci, ei, _ = oracle.batch(oracle.I64, qc, w.reads.offsets, codes)
    assert np.all(np.abs(ei[on] - w.reads.end_true[on]) <= 10)


def test_noise_spread_scales_each_reads_noise_and_changes_nothing_else():
    # per-read noise between 1x and spread x (log-uniform), from a generator
    # of its own: spread 1 reproduces the default reads exactly, and a spread
    # changes only the noise of the genomic reads, not which reads are on
    # target or where they start
    genome = synth.make_genome(20_000, 5)
    table = synth.make_level_table()
    L = np.full(64, 300)
    base = synth.simulate_reads(genome, table, L, 0.5, 11)
    same = synth.simulate_reads(genome, table, L, 0.5, 11, noise_spread=1.0)
    assert np.array_equal(base.values, same.values)
    wide = synth.simulate_reads(genome, table, L, 0.5, 11, noise_spread=4.0)
    assert np.array_equal(base.on_target, wide.on_target)
    assert np.array_equal(base.start, wide.start) and np.array_equal(base.strand, wide.strand)
    # same strand, start and dwell draws: the difference of two reads is the
    # difference of their noise, whose sd ratio is the read's multiplier
    ratios = []
    for r in np.nonzero(base.on_target)[0]:
        a, b = base.offsets[r], base.offsets[r + 1]
        d = (wide.values[a:b].astype(np.float64) - base.values[a:b]) / synth.NOISE_SD_PA
        ratios.append(d.std())
    ratios = np.array(ratios)
    # (mult - 1) x N(0, 1): between 0 and 3 in sd, spread over the range
    assert ratios.min() < 0.5 and ratios.max() > 2.0 and ratios.max() < 3.3
    with np.testing.assert_raises(ValueError):
        synth.simulate_reads(genome, table, L, 0.5, 11, noise_spread=0.5)
