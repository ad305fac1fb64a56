"""The batch step (query preparation + alignment), and the same step from raw
samples (event detection + preparation + alignment), captured in a HIP
graph: every replay must equal the eager result, with eager work and host
synchronisation between the replays."""
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


@pytest.mark.parametrize("bands", [1, 2])
def test_batch_step_in_a_graph(bands):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    w = synth.workload(2, nq=96)
    z, codes, _ = oracle.prepare_reference(w.genome, w.table, w.k)
    ref = sd.Reference(torch.from_numpy(codes).to(dev))
    plan = sd.Plan(w.reads.offsets, sd.I16)
    plan.set_config(strip=16, chains=1, waves_per_cu=4 * bands, bands=bands)
    raw = torch.from_numpy(w.reads.values).to(dev)
    offs = torch.from_numpy(w.reads.offsets).to(dev)
    cost = torch.empty(w.reads.nq, dtype=torch.int32, device=dev)
    end = torch.empty(w.reads.nq, dtype=torch.int32, device=dev)

    def step():
        _, q, _ = sd.prepare_queries(raw, offs, 64.0)
        sd.align_batch(ref, plan, q, cost, end)

    note(f"eager bands={bands}")
    step()
    torch.cuda.synchronize()
    want = (cost.cpu().numpy().copy(), end.cpu().numpy().copy())
    qz, qc, _ = oracle.prepare_queries(w.reads.values, w.reads.offsets)
    idx = np.arange(0, w.reads.nq, 12)
    wc, we, _ = oracle.batch(oracle.I64, qc, w.reads.offsets, codes, index=idx)
    assert np.array_equal(want[0][idx], wc.astype(np.int64))
    assert np.array_equal(want[1][idx], we)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream before capture
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    note("capture")
    with torch.cuda.graph(g):
        step()
    for k in range(4):
        cost.fill_(-1)
        end.fill_(-1)
        torch.cuda.synchronize()
        note(f"replay {k}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), want[0]), k
        assert np.array_equal(end.cpu().numpy(), want[1]), k
        step()  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), want[0]), k
    plan.close()
    ref.close()


def test_raw_samples_to_alignment_in_a_graph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import events as oev
    dev = torch.device("cuda:0")
    g_np = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    table = synth.make_level_table()
    raw = synth.simulate_raw(g_np, table, 64, 320, 0.5, 808)
    _, codes, _ = oracle.prepare_reference(g_np, table, synth.K)
    ref = sd.Reference(torch.from_numpy(codes).to(dev))
    x = torch.from_numpy(raw.values).to(dev)
    xo = torch.from_numpy(raw.offsets).to(dev)
    eo_np = np.arange(65, dtype=np.int64) * 250
    eo = torch.from_numpy(eo_np).to(dev)
    plan = sd.Plan(eo_np, sd.I16)
    plan.set_config(strip=16, chains=1, waves_per_cu=4, bands=1)
    ev = torch.empty((64, 250), dtype=torch.float32, device=dev)
    cnt = torch.empty(64, dtype=torch.int32, device=dev)
    cost = torch.empty(64, dtype=torch.int32, device=dev)
    end = torch.empty(64, dtype=torch.int32, device=dev)

    def step():
        sd.detect_events(x, xo, 50, 250, events=ev, counts=cnt)
        _, q, _ = sd.prepare_queries(ev.reshape(-1), eo, 64.0)
        sd.align_batch(ref, plan, q, cost, end)

    note("eager raw pipeline")
    step()
    torch.cuda.synchronize()
    assert bool((cnt == 250).all())
    want = (cost.cpu().numpy().copy(), end.cpu().numpy().copy())
    # the oracle on a sample of the reads
    for r in (0, 17, 63):
        e = oev.query_events(raw.values[raw.offsets[r]:raw.offsets[r + 1]], 50, 250)
        qo, _ = oracle.quantize(oracle.znorm(e), 64.0)
        assert (int(want[0][r]), int(want[1][r])) == oracle.sdtw_i64(qo, codes), r
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    note("capture raw pipeline")
    with torch.cuda.graph(g):
        step()
    for k in range(4):
        cost.fill_(-1)
        end.fill_(-1)
        ev.fill_(0)
        torch.cuda.synchronize()
        note(f"replay {k}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), want[0]), k
        assert np.array_equal(end.cpu().numpy(), want[1]), k
        step()
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), want[0]), k
    plan.close()
    ref.close()
