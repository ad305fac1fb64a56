"""Seeded synthetic inputs for sDTW Read Until workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no step of the alignment method: it only simulates what a nanopore run
would hand to the method, in raw units.

* ``make_genome``       -- uniform random bases A/C/G/T coded 0..3.
* ``make_level_table``  -- a stand-in pore model: one expected current per
  6-mer, drawn i.i.d. from N(90, 12) pA (the real R9.4 table is not
  available; the section 5.3 datasets are not available either).
* ``simulate_raw``      -- raw sample streams in pA (30 adaptor levels, then
  one level per base, each held for 4-14 samples, N(0, 1.5 pA) sample
  noise), the input of event detection.
* ``simulate_reads``    -- event streams in pA.  An on-target read picks a
  strand and a start, walks the strand's bases 5'->3' and emits the pore
  model's level of each successive 6-mer 1, 2 or 3 times (uniform), each
  emission with additive N(0, 0.3 x 12 pA) noise.  An off-target read is
  i.i.d. N(90, 12) pA, or (``off_genome``) the same pore simulation run on
  another genome, the harder case of reads from a background organism.
  ``noise_spread`` gives each read its own noise level (1x to spread x,
  log-uniform), as reads from different pores would have.
  Lengths follow the workload.

The sizes mirror the paper's workloads (Table 2: the 29,903-base SARS-CoV-2
genome and 250-event queries, section 4.1), which stand in for the missing
datasets.  Everything is deterministic in its seed (NumPy PCG64).

Workload presets (``workload(c)``):
  0  one on-target read, M=250, 29,903-base genome (seed 29903)
  1  4,096 reads, M=250, 50% on-target
  2  8,192 reads, M ~ U{100..2000}, 70% on-target
  3  1,024 reads, M ~ U{250..500}, 50% on-target, 5,000,000-base genome
  4  streaming: 512 channels of 400-event chunks (see ``channel_reads``)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

K = 6
LEVEL_MEAN_PA = 90.0
LEVEL_SD_PA = 12.0
NOISE_SD_PA = 0.3 * LEVEL_SD_PA  # N(0, 0.3) in reference z-units
SMALL_GENOME = 29_903
LARGE_GENOME = 5_000_000
TABLE_SEED = 6


def make_genome(length: int, seed: int) -> np.ndarray:
    """Uniform random bases coded A=0, C=1, G=2, T=3 (uint8)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4, size=int(length), dtype=np.uint8)


def make_level_table(k: int = K, seed: int = TABLE_SEED) -> np.ndarray:
    """Stand-in pore model: 4**k levels ~ N(90, 12) pA in k-mer index order."""
    rng = np.random.default_rng(seed)
    return rng.normal(LEVEL_MEAN_PA, LEVEL_SD_PA, size=4 ** k).astype(np.float32)


def _pore_current(bases: np.ndarray, table: np.ndarray, k: int) -> np.ndarray:
    """Expected current of each successive k-mer of a strand (pore simulation)."""
    n = bases.size - k + 1
    idx = np.zeros(n, dtype=np.int64)
    for m in range(k):
        idx = idx * 4 + bases[m:m + n].astype(np.int64)
    return table[idx]


@dataclass
class Reads:
    values: np.ndarray      # float32, concatenated raw events (pA)
    offsets: np.ndarray     # int64, nq + 1
    on_target: np.ndarray   # bool, per read
    strand: np.ndarray      # int8: 0 forward, 1 reverse, -1 off-target
    start: np.ndarray       # int64: first k-mer index on the strand (-1 off-target)
    end_true: np.ndarray    # int64: index of the last emitted k-mer in the
                            # forward||reverse concatenation (-1 off-target)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def nq(self) -> int:
        return self.offsets.size - 1


def _genomic_events(genome: np.ndarray, table: np.ndarray, M: int, k: int,
                    noise_sd: float, rng) -> tuple[np.ndarray, int, int, int]:
    """M events of a random strand and start of ``genome``: (events, strand,
    start, k-mers emitted - 1)."""
    nk = genome.size - k + 1
    s = int(rng.integers(0, 2))
    p = int(rng.integers(0, nk - M + 1))  # M k-mers always fit
    reps = rng.integers(1, 4, size=M)
    strand_bases = genome if s == 0 else (3 - genome[::-1]).astype(np.uint8)
    levels = _pore_current(strand_bases[p:p + M + k - 1], table, k)
    ev = np.repeat(levels, reps)[:M]
    ev = ev + rng.normal(0.0, noise_sd, size=M)
    used = int(np.searchsorted(np.cumsum(reps), M))
    return ev.astype(np.float32), s, p, used


def simulate_reads(genome: np.ndarray, table: np.ndarray, lengths,
                   frac_on: float, seed: int, k: int = K,
                   noise_sd: float = NOISE_SD_PA,
                   off_genome: np.ndarray | None = None,
                   noise_spread: float = 1.0) -> Reads:
    """Raw event streams for reads of the given lengths (see module doc).

    ``off_genome``: off-target reads are drawn from this other genome the
    way on-target reads are drawn from ``genome`` (pore signal of a random
    strand and start), instead of i.i.d. N(90, 12) pA values.

    ``noise_spread`` > 1: every read's event noise is ``noise_sd`` times
    spread**u, u ~ U(0, 1) per read (log-uniform between 1x and spread x),
    drawn from a generator of its own so that the rest of the draws, and the
    reads of spread 1, stay the same."""
    rng = np.random.default_rng(seed)
    if noise_spread < 1.0:
        raise ValueError("noise_spread must be >= 1")
    mult = np.ones(len(np.atleast_1d(lengths)))
    if noise_spread != 1.0:
        mult = noise_spread ** np.random.default_rng(seed + 104729).random(mult.size)
    lengths = np.asarray(lengths, dtype=np.int64)
    nq = lengths.size
    offsets = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    values = np.empty(int(offsets[-1]), dtype=np.float32)
    on = rng.random(nq) < frac_on
    strand = np.full(nq, -1, dtype=np.int8)
    start = np.full(nq, -1, dtype=np.int64)
    end_true = np.full(nq, -1, dtype=np.int64)
    nk = genome.size - k + 1
    nk_off = -1 if off_genome is None else off_genome.size - k + 1
    for r in range(nq):
        M = int(lengths[r])
        a, b = int(offsets[r]), int(offsets[r + 1])
        if on[r] and nk >= M:
            values[a:b], s, p, used = _genomic_events(genome, table, M, k,
                                                      noise_sd * float(mult[r]), rng)
            strand[r] = s
            start[r] = p
            end_true[r] = s * nk + p + used
        elif nk_off >= M:
            on[r] = False
            values[a:b] = _genomic_events(off_genome, table, M, k, noise_sd * float(mult[r]),
                                          rng)[0]
        else:
            on[r] = False
            values[a:b] = rng.normal(LEVEL_MEAN_PA, LEVEL_SD_PA, size=M).astype(np.float32)
    return Reads(values, offsets, on, strand, start, end_true)


SAMPLE_NOISE_PA = 1.5          # per-sample noise of raw current
DWELL_SAMPLES = (4, 14)        # samples per base: uniform, mean 9 (4 kHz at 450 b/s)
ADAPTOR_LEVELS = 30            # adaptor levels before the read's own bases (about 50
                               # detected events: the detector cuts ~1.7 events per level)


@dataclass
class RawReads:
    values: np.ndarray      # float32, concatenated raw samples (pA)
    offsets: np.ndarray     # int64, nreads + 1
    on_target: np.ndarray   # bool
    strand: np.ndarray      # int8: 0 forward, 1 reverse, -1 off-target
    start: np.ndarray       # int64: first k-mer index on the strand (-1 off-target)
    levels: list            # per read: the expected level of every event (adaptor first)

    @property
    def nreads(self) -> int:
        return self.offsets.size - 1


def simulate_raw(genome: np.ndarray, table: np.ndarray, nreads: int, bases: int,
                 frac_on: float, seed: int, k: int = K, adaptor: int = ADAPTOR_LEVELS,
                 dwell=DWELL_SAMPLES, noise_sd: float = SAMPLE_NOISE_PA,
                 off_genome: np.ndarray | None = None) -> RawReads:
    """Raw sample streams, the input of event detection: ``adaptor`` levels
    drawn from N(90, 12) pA, then one level per base of the read (the pore
    model's level of each successive k-mer of a random strand and start of
    ``genome``, or of ``off_genome``, or N(90, 12) pA for off-target reads
    without one); every level lasts a uniform number of samples in
    ``dwell`` and every sample carries N(0, noise_sd) pA noise."""
    rng = np.random.default_rng(seed)
    on = rng.random(nreads) < frac_on
    strand = np.full(nreads, -1, dtype=np.int8)
    start = np.full(nreads, -1, dtype=np.int64)
    chunks, levels = [], []
    for r in range(nreads):
        lv = [rng.normal(LEVEL_MEAN_PA, LEVEL_SD_PA, size=adaptor)]
        src = genome if on[r] else off_genome
        if src is not None and src.size - k + 1 >= bases:
            s = int(rng.integers(0, 2))
            p = int(rng.integers(0, src.size - k + 1 - bases + 1))
            strand_bases = src if s == 0 else (3 - src[::-1]).astype(np.uint8)
            lv.append(_pore_current(strand_bases[p:p + bases + k - 1], table, k))
            if on[r]:
                strand[r], start[r] = s, p
        else:
            on[r] = False
            lv.append(rng.normal(LEVEL_MEAN_PA, LEVEL_SD_PA, size=bases))
        lv = np.concatenate(lv).astype(np.float64)
        reps = rng.integers(dwell[0], dwell[1] + 1, size=lv.size)
        x = np.repeat(lv, reps) + rng.normal(0.0, noise_sd, size=int(reps.sum()))
        chunks.append(x.astype(np.float32))
        levels.append(lv.astype(np.float32))
    offsets = np.zeros(nreads + 1, dtype=np.int64)
    np.cumsum([c.size for c in chunks], out=offsets[1:])
    return RawReads(np.concatenate(chunks), offsets, on, strand, start, levels)


@dataclass
class Workload:
    name: str
    genome: np.ndarray
    table: np.ndarray
    reads: Reads
    k: int = K


def workload(c: int, nq: int | None = None) -> Workload:
    """Seeded preset c in {0,1,2,3}; ``nq`` optionally truncates the read count
    (the first nq reads of the full preset, same seed, same values)."""
    if c in (0, 1, 2):
        genome = make_genome(SMALL_GENOME, SMALL_GENOME)
    elif c == 3:
        genome = make_genome(LARGE_GENOME, LARGE_GENOME)
    else:
        raise ValueError(f"no batch preset {c}")
    table = make_level_table()
    seed = 1000 + c
    rng = np.random.default_rng(seed + 500)
    if c == 0:
        lengths, frac, name = np.array([250]), 1.0, "single read M=250 vs 29,903-base genome"
    elif c == 1:
        lengths, frac, name = np.full(4096, 250), 0.5, "4096 reads M=250 vs 29,903-base genome"
    elif c == 2:
        lengths, frac, name = rng.integers(100, 2001, size=8192), 0.7, \
            "8192 reads M~U[100,2000] vs 29,903-base genome"
    else:
        lengths, frac, name = rng.integers(250, 501, size=1024), 0.5, \
            "1024 reads M~U[250,500] vs 5,000,000-base genome"
    reads = simulate_reads(genome, table, lengths, frac, seed)
    if nq is not None and nq < reads.nq:
        reads = take(reads, np.arange(nq))
    return Workload(name, genome, table, reads)


def take(reads: Reads, idx) -> Reads:
    """Sub-batch of reads (in the order of ``idx``)."""
    idx = np.asarray(idx, dtype=np.int64)
    lens = reads.lengths[idx]
    offs = np.zeros(idx.size + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    vals = np.concatenate([reads.values[reads.offsets[i]:reads.offsets[i + 1]]
                           for i in idx]) if idx.size else np.zeros(0, np.float32)
    return Reads(vals.astype(np.float32), offs, reads.on_target[idx],
                 reads.strand[idx], reads.start[idx], reads.end_true[idx])


def csr(arrays) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate a list of 1-D arrays into (values, int64 offsets)."""
    lens = np.array([len(a) for a in arrays], dtype=np.int64)
    offs = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    vals = np.concatenate(arrays) if len(arrays) else np.zeros(0)
    return vals, offs
