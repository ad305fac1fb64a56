"""Parity at the full batch sizes, in the launch configuration the benchmark
times (library preparation of the reference and of the reads on the device,
then the launch shape picked by the library's autotuner on the batch):

* workload 1: 4,096 reads of 250 events against 59,796 columns;
* workload 2: 8,192 reads of 100-2,000 events against 59,796 columns;
* workload 3: 1,024 reads of 250-500 events against 9,999,990 columns.

First the device preparation (section 4.1) must equal the oracle's bit for
bit: reference z values and int16 codes, read z values and codes.  Then:

* workloads 1 and 2, every read (workload 2's float32 check in two halves):
  int16 bit-exact against the exact integer
  oracle; float32 bit-exact against the float32-sequenced oracle; and within
  1e-5 relative of the float64 oracle, whose last row must accept the GPU's
  end where the two ends differ (every read of workload 1, a seeded sample
  of 1,024 reads of workload 2);
* workload 3, a seeded sample of 64 reads plus the shortest and the longest
  (66 reads), both formats, the float64 gate on 8 of them;
* every on-target read ends within 10 columns of where it was simulated from.

The oracle runs on at most 16 host threads.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.load_library()
    return torch.device("cuda:0")


def chain(dev, w, dtype):
    """The product path: reference and reads prepared on the device, the plan
    autotuned on the batch, one batched alignment.  Returns the prepared
    arrays (host copies) and (cost, end)."""
    g = torch.from_numpy(w.genome).to(dev)
    t = torch.from_numpy(w.table).to(dev)
    zr, cr, nsat_r = sd.prepare_reference(g, t, w.k, 64.0)
    raw = torch.from_numpy(w.reads.values).to(dev)
    offs_dev = torch.from_numpy(w.reads.offsets).to(dev)
    zq, cq, nsat_q = sd.prepare_queries(raw, offs_dev, 64.0)
    ref = sd.Reference(cr if dtype == sd.I16 else zr)
    plan = sd.Plan(w.reads.offsets, dtype)
    q = cq if dtype == sd.I16 else zq
    cfg = sd.autotune(ref, plan, q)
    cost, end = sd.align_batch(ref, plan, q)
    torch.cuda.synchronize()
    out = {"zr": zr.cpu().numpy(), "cr": cr.cpu().numpy(), "nsat_r": int(nsat_r.item()),
           "zq": zq.cpu().numpy(), "cq": cq.cpu().numpy(), "nsat_q": int(nsat_q.item()),
           "cost": cost.cpu().numpy(), "end": end.cpu().numpy(), "cfg": cfg}
    plan.close()
    ref.close()
    return out


def check_prep(got, want):
    """Device preparation equals the oracle's bit for bit."""
    z, codes, nsat, qz, qc, qnsat = want
    assert np.array_equal(got["zr"].view(np.uint32), z.view(np.uint32))
    assert np.array_equal(got["cr"], codes) and got["nsat_r"] == nsat
    assert np.array_equal(got["zq"].view(np.uint32), qz.view(np.uint32))
    assert np.array_equal(got["cq"], qc) and got["nsat_q"] == qnsat


def run_oracle(kind, q, offs, ref, index):
    """oracle.batch over `index` in pieces of about 5e10 cells, printing a
    line after each piece (a long check keeps reporting progress)."""
    lens = (offs[index + 1] - offs[index]).astype(np.float64) * ref.size
    cut = np.searchsorted(np.cumsum(lens), np.arange(5e10, lens.sum(), 5e10))
    cost, end = [], []
    t0 = time.perf_counter()
    for part in np.split(index, cut):
        if part.size == 0:
            continue
        c, e, _ = oracle.batch(kind, q, offs, ref, index=part, nthreads=THREADS)
        cost.append(c)
        end.append(e)
        note(f"    oracle {['int64', 'float32', 'float64'][kind]}: "
             f"{sum(x.size for x in cost)}/{index.size} reads, {time.perf_counter() - t0:.1f} s")
    return np.concatenate(cost), np.concatenate(end)


def check_i16(got, q, offs, ref, index):
    want_c, want_e = run_oracle(oracle.I64, q, offs, ref, index)
    gc, ge = got["cost"][index].astype(np.int64), got["end"][index]
    bad = np.nonzero((gc != want_c.astype(np.int64)) | (ge != want_e))[0]
    assert bad.size == 0, (index[bad][:5], gc[bad][:5], ge[bad][:5], want_c[bad][:5],
                           want_e[bad][:5])
    return index.size


def check_f32(got, q, offs, ref, index, f64_index):
    want_c, want_e = run_oracle(oracle.F32, q, offs, ref, index)
    gc, ge = got["cost"][index].astype(np.float64), got["end"][index]
    bad = np.nonzero((gc != want_c) | (ge != want_e))[0]
    assert bad.size == 0, (index[bad][:5], gc[bad][:5], ge[bad][:5], want_c[bad][:5],
                           want_e[bad][:5])
    # float64 gate: cost within 1e-5 relative; where the ends differ, the
    # float64 last row at the GPU's end within the same bound
    c64, e64 = run_oracle(oracle.F64, q, offs, ref, f64_index)
    g64c, g64e = got["cost"][f64_index].astype(np.float64), got["end"][f64_index]
    rel = np.abs(g64c - c64) / np.maximum(c64, 1e-30)
    assert rel.max() <= 1e-5, (f64_index[np.argmax(rel)], rel.max())
    differ = np.nonzero(g64e != e64)[0]
    for t in differ:
        r = int(f64_index[t])
        c, _, lr = oracle.sdtw_f64(q[offs[r]:offs[r + 1]], ref, lastrow=True)
        assert lr[g64e[t]] <= c * (1 + 1e-5) + 1e-30, (r, g64e[t], e64[t])
    return index.size, f64_index.size, differ.size


def check_on_target(ends, reads):
    on = reads.on_target
    d = np.abs(ends[on].astype(np.int64) - reads.end_true[on])
    assert np.mean(d <= 10) > 0.99, (np.mean(d <= 10), np.sort(d)[-5:])


def oracle_prep(w):
    z, codes, nsat = oracle.prepare_reference(w.genome, w.table, w.k)
    qz, qc, qnsat = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    return z, codes, nsat, qz, qc, qnsat


@pytest.fixture(scope="module")
def workload1():
    w = synth.workload(1)
    return w, oracle_prep(w)


@pytest.fixture(scope="module")
def workload2():
    w = synth.workload(2)
    return w, oracle_prep(w)


@pytest.fixture(scope="module")
def workload3():
    w = synth.workload(3)
    return w, oracle_prep(w)


def workload3_sample(w):
    lens = w.reads.lengths
    rnd = np.random.default_rng(23).choice(w.reads.nq, size=64, replace=False)
    return np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens)], rnd]))


@pytest.mark.parametrize("wl", ["workload1", "workload2"])
def test_every_read_int16(dev, wl, request):
    w, want = request.getfixturevalue(wl)
    note(f"{w.name}, int16: device preparation, autotuned launch, every read")
    got = chain(dev, w, sd.I16)
    note(f"  launch shape {got['cfg']}")
    check_prep(got, want)
    n = check_i16(got, want[4], w.reads.offsets, want[1], np.arange(w.reads.nq))
    note(f"  {n} of {w.reads.nq} reads bit-exact against the int64 oracle")
    check_on_target(got["end"], w.reads)


@pytest.mark.parametrize("wl,part", [("workload1", None), ("workload2", 0), ("workload2", 1)])
def test_every_read_float32(dev, wl, part, request):
    # workload 2 is checked in two halves (reads of even, then odd index), so
    # that each test stays within a couple of minutes of oracle time
    w, want = request.getfixturevalue(wl)
    note(f"{w.name}, float32: device preparation, autotuned launch, every read "
         f"{'' if part is None else ('of even index' if part == 0 else 'of odd index')}")
    got = chain(dev, w, sd.F32)
    note(f"  launch shape {got['cfg']}")
    check_prep(got, want)
    every = np.arange(w.reads.nq)
    # float64 on every read of workload 1; on a seeded sample of 1,024 reads
    # of workload 2 (all 8,192 would double the check's time)
    f64 = every if w.reads.nq <= 4096 else np.sort(
        np.random.default_rng(25).choice(w.reads.nq, size=1024, replace=False))
    if part is not None:
        every = every[every % 2 == part]
        f64 = f64[f64 % 2 == part]
    n, n64, nd = check_f32(got, want[3], w.reads.offsets, want[0], every, f64)
    note(f"  {n} reads bit-exact against the float32 oracle; {n64} within 1e-5 of float64 "
         f"({nd} ends differ from float64's, each accepted by its last row)")
    check_on_target(got["end"], w.reads)


def test_workload3_int16_sample(dev, workload3):
    w, want = workload3
    note(f"{w.name}, int16: device preparation, autotuned launch")
    got = chain(dev, w, sd.I16)
    note(f"  launch shape {got['cfg']}")
    check_prep(got, want)
    n = check_i16(got, want[4], w.reads.offsets, want[1], workload3_sample(w))
    note(f"  {n} sampled reads (seed 23, shortest and longest included) bit-exact")
    check_on_target(got["end"], w.reads)


def test_workload3_float32_sample(dev, workload3):
    w, want = workload3
    note(f"{w.name}, float32: device preparation, autotuned launch")
    got = chain(dev, w, sd.F32)
    note(f"  launch shape {got['cfg']}")
    check_prep(got, want)
    sample = workload3_sample(w)
    n, n64, nd = check_f32(got, want[3], w.reads.offsets, want[0], sample, sample[:8])
    note(f"  {n} sampled reads bit-exact against the float32 oracle; {n64} within 1e-5 "
         f"of float64")
    check_on_target(got["end"], w.reads)
