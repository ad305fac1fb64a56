"""Read Until server: every result it serves equals the oracle's on the read's
prefix (normalised with its first chunk), whatever the mix it ran in."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")


def test_served_results_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_07340_amd import server as srv
    dev = torch.device("cuda:0")
    table = synth.make_level_table()
    genome = synth.make_genome(synth.SMALL_GENOME, synth.SMALL_GENOME)
    rd = synth.simulate_reads(genome, table, np.full(48, 2000), 0.5, 91)
    raws = [rd.values[rd.offsets[r]:rd.offsets[r + 1]] for r in range(48)]
    # the reference codes come from the oracle, so that every input of the
    # check below is independent of the library
    z, codes, _ = oracle.prepare_reference(genome, table, 6)
    targets = [srv.Target("small", sd.Reference(torch.from_numpy(codes).to(dev)), raws,
                          np.asarray(rd.on_target, bool))]
    rec = []
    server = srv.ReadUntilServer(targets, srv.ServerConfig(channels=24), record=rec)
    taus = server.calibrate(n_each=16)
    res = server.run(2.0, 0.5)
    assert res["decisions"] > 20 and res["decision_accuracy"] > 0.9, res
    assert rec, "nothing served"
    rng = np.random.default_rng(0)
    for t, pi, rows, cost, end in [rec[i] for i in rng.choice(len(rec), 24, replace=False)]:
        raw = raws[pi]
        mean, sdv = oracle.zstats(raw[:400])
        q, _ = oracle.quantize(oracle.zapply(raw[:rows], mean, sdv), 64.0)
        assert oracle.sdtw_i64(q, codes) == (cost, end), (pi, rows)
    targets[0].ref.close()
