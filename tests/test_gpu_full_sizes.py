"""Parity at the full batch sizes, in the launch configuration the benchmark
times (the launch shape picked by the library's autotuner on the batch):

* workload 2: 8,192 reads of 100-2,000 events against 59,796 columns;
* workload 3: 1,024 reads of 250-500 events against 9,999,990 columns.

The oracle cannot run every read of these batches in a test, so a seeded
sample of reads is computed one by one (int16: bit-exact against the exact
integer oracle; float32: bit-exact against the float32-sequenced oracle and
within 1e-5 relative of float64), and every on-target read is checked
against a property that holds at any size: it ends within 10 columns of the
position it was simulated from (a sample of each workload's on-target reads
ends within 2 columns in the oracle).
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


def tuned_batch(dev, ref_np, q_np, offs, dtype):
    """Autotune the plan on the batch, then align it (as the benchmark does)."""
    ref = sd.Reference(torch.from_numpy(np.ascontiguousarray(ref_np)).to(dev))
    plan = sd.Plan(offs, dtype)
    q = torch.from_numpy(np.ascontiguousarray(q_np)).to(dev)
    cfg = sd.autotune(ref, plan, q)
    cost, end = sd.align_batch(ref, plan, q)
    torch.cuda.synchronize()
    out = cost.cpu().numpy(), end.cpu().numpy()
    plan.close()
    ref.close()
    return out, cfg


def check_sample_i16(got, q, offs, ref, index):
    want_c, want_e, _ = oracle.batch(oracle.I64, q, offs, ref, index=index)
    gc, ge = got[0][index].astype(np.int64), got[1][index]
    bad = np.nonzero((gc != want_c.astype(np.int64)) | (ge != want_e))[0]
    assert bad.size == 0, (index[bad], gc[bad], ge[bad], want_c[bad], want_e[bad])


def check_sample_f32(got, q, offs, ref, index, f64_reads):
    want_c, want_e, _ = oracle.batch(oracle.F32, q, offs, ref, index=index)
    gc, ge = got[0][index].astype(np.float64), got[1][index]
    bad = np.nonzero((gc != want_c) | (ge != want_e))[0]
    assert bad.size == 0, (index[bad], gc[bad], ge[bad], want_c[bad], want_e[bad])
    for r in f64_reads:
        c64, _, lr = oracle.sdtw_f64(q[offs[r]:offs[r + 1]], ref, lastrow=True)
        c, e = float(got[0][r]), int(got[1][r])
        assert abs(c - c64) <= 1e-5 * max(c64, 1e-30), (r, c, c64)
        assert lr[e] <= c64 * (1 + 1e-5) + 1e-30, (r, e)


def check_on_target(ends, reads):
    on = reads.on_target
    d = np.abs(ends[on].astype(np.int64) - reads.end_true[on])
    assert np.mean(d <= 10) > 0.99, (np.mean(d <= 10), np.sort(d)[-5:])


@pytest.fixture(scope="module")
def workload2():
    w = synth.workload(2)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    return w, z, codes, qz, qc


@pytest.fixture(scope="module")
def workload3():
    w = synth.workload(3)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    return w, z, codes, qz, qc


def test_full_workload2_int16(dev, workload2):
    w, _, codes, _, qc = workload2
    offs = w.reads.offsets
    note(f"workload 2 int16: {w.reads.nq} reads vs {codes.size} columns, autotuned")
    got, cfg = tuned_batch(dev, codes, qc, offs, sd.I16)
    note(f"  launch shape {cfg}")
    sample = np.random.default_rng(21).choice(w.reads.nq, size=32, replace=False)
    check_sample_i16(got, qc, offs, codes, sample)
    check_on_target(got[1], w.reads)


def test_full_workload2_float32(dev, workload2):
    w, z, _, qz, _ = workload2
    offs = w.reads.offsets
    note(f"workload 2 float32: {w.reads.nq} reads vs {z.size} columns, autotuned")
    got, cfg = tuned_batch(dev, z, qz, offs, sd.F32)
    note(f"  launch shape {cfg}")
    sample = np.random.default_rng(22).choice(w.reads.nq, size=12, replace=False)
    check_sample_f32(got, qz, offs, z, sample, f64_reads=sample[:3])
    check_on_target(got[1], w.reads)


def test_full_workload3_int16(dev, workload3):
    w, _, codes, _, qc = workload3
    offs = w.reads.offsets
    note(f"workload 3 int16: {w.reads.nq} reads vs {codes.size} columns, autotuned")
    got, cfg = tuned_batch(dev, codes, qc, offs, sd.I16)
    note(f"  launch shape {cfg}")
    # the shortest and the longest read and four drawn at random
    lens = w.reads.lengths
    rnd = np.random.default_rng(23).choice(w.reads.nq, size=4, replace=False)
    sample = np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens)], rnd]))
    check_sample_i16(got, qc, offs, codes, sample)
    check_on_target(got[1], w.reads)


def test_full_workload3_float32(dev, workload3):
    w, z, _, qz, _ = workload3
    offs = w.reads.offsets
    note(f"workload 3 float32: {w.reads.nq} reads vs {z.size} columns, autotuned")
    got, cfg = tuned_batch(dev, z, qz, offs, sd.F32)
    note(f"  launch shape {cfg}")
    lens = w.reads.lengths
    rnd = np.random.default_rng(24).choice(w.reads.nq, size=2, replace=False)
    sample = np.unique(np.concatenate([[np.argmin(lens)], rnd]))
    check_sample_f32(got, qz, offs, z, sample, f64_reads=[int(np.argmin(lens))])
    check_on_target(got[1], w.reads)
