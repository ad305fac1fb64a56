"""Host logic of the Read Until server's decision rules (no GPU)."""
import numpy as np
import pytest

from paper_2211_07340_amd import server as srv


def test_mapq_range_and_monotone():
    best = np.array([0, 0, 10, 10, 10, 50, 7])
    second = np.array([0, 5, 10, 20, 40, 100, np.iinfo(np.int32).max])
    q = srv.mapq(best, second)
    # equal costs: no information; best 0: perfectly separated
    assert q.tolist() == [0, 60, 0, 30, 45, 30, 60]
    assert srv.mapq(3.0, float("inf")) == 60
    # scale-free: the same read as int16 codes or float32 values
    assert srv.mapq(12.5, 25.0) == srv.mapq(800, 1600) == 30
    # monotone in the gap
    s = np.linspace(10, 1000, 200)
    assert np.all(np.diff(srv.mapq(np.full(200, 10.0), s)) >= 0)


class _T:
    def __init__(self):
        self.tau, self.q_min = 0.3, 20.0


class _R:
    def __init__(self, rows):
        self.target, self.rows = 0, rows


def _server(decision):
    s = srv.ReadUntilServer.__new__(srv.ReadUntilServer)
    s.cfg = srv.ServerConfig(decision=decision, min_reject_events=800, max_events=2000)
    s.targets = [_T()]
    return s


@pytest.mark.parametrize("decision", ["cost", "mapq"])
def test_decide(decision):
    s = _server(decision)
    def good(rows):  # 0.2 z-units per event; q = 54
        return (0.2 * 64 * rows, 1e9) if decision == "cost" else (100, 1000)

    def bad(rows):   # 0.5 z-units per event; q = 1
        return (0.5 * 64 * rows, 1e9) if decision == "cost" else (990, 1000)

    assert s._decide(_R(400), *good(400)) == "keep"
    assert s._decide(_R(400), *bad(400)) is None          # too early to reject
    assert s._decide(_R(800), *bad(800)) == "reject"
    assert s._decide(_R(2000), *bad(2000)) == "reject"
    assert s._decide(_R(2000), *good(2000)) == "keep"


def test_rule_names_checked():
    with pytest.raises(ValueError):
        srv.ReadUntilServer.__init__(srv.ReadUntilServer.__new__(srv.ReadUntilServer), [],
                                     srv.ServerConfig(decision="vote"))
