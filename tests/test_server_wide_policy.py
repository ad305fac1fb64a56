"""Which extension the server issues for a batch (CPU only): one batched
launch (sdtw_stream_extend), or for at most a target's ``wide_max`` chunks
one whole-device call per chunk (sdtw_stream_extend_wide), on the batch's
HIP stream, or with ``wide_streams=2`` alternating between it and the
target's second one, which waits for the batch's stream first and is
waited for at the end.  The binding calls are replaced by recorders; no
device is touched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2211_07340_amd import binding as sd  # noqa: E402
from paper_2211_07340_amd import server as srv  # noqa: E402


class FakeStream:
    def __init__(self, name, log):
        self.name, self.log = name, log

    def wait_stream(self, other):
        self.log.append(("wait", self.name, other.name))


class Handle:
    def __init__(self, rows):
        self.rows = rows


class Target:
    def __init__(self, wide_max, log, dtype=sd.I16):
        self.wide_max = wide_max
        self.wide_aux = FakeStream("aux", log)
        self.ref = type("R", (), {"dtype": dtype})()


class Server(srv.ReadUntilServer):
    def __init__(self, cfg=None):  # no device set-up
        self.cfg = cfg or srv.ServerConfig()
        self.torch = torch
        self._loop = None


@pytest.fixture
def calls(monkeypatch):
    log = []

    def wide(h, chunk, cols=0, cost=None, end=None, stream=None):
        log.append(("wide", id(h), int(chunk.numel()), stream.name))
        cost.fill_(chunk.numel())
        end.fill_(-chunk.numel())

    def batched(handles, codes, offs, stream=None):
        log.append(("batch", len(handles), stream.name))
        k = len(handles)
        return torch.zeros(k, dtype=torch.int32), torch.zeros(k, dtype=torch.int32)

    monkeypatch.setattr(sd, "stream_extend_wide", wide)
    monkeypatch.setattr(sd, "stream_extend", batched)
    return log


def _batch(lens, rows=0):
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    codes = torch.zeros(int(offs[-1]), dtype=torch.int16)
    return [Handle(rows) for _ in lens], codes, offs


def test_small_batches_go_over_the_whole_device(calls):
    t = Target(4, calls)
    handles, codes, offs = _batch([400, 300, 200])
    cost, end = Server()._extend(t, handles, codes, offs, FakeStream("hs", calls))
    assert [(c[0], c[2], c[3]) for c in calls] == [("wide", 400, "hs"), ("wide", 300, "hs"),
                                                   ("wide", 200, "hs")]
    assert cost.tolist() == [400, 300, 200] and end.tolist() == [-400, -300, -200]


def test_small_batches_on_two_streams(calls):
    t = Target(4, calls)
    hs = FakeStream("hs", calls)
    handles, codes, offs = _batch([400, 300, 200])
    cost, end = Server(srv.ServerConfig(wide_streams=2))._extend(t, handles, codes, offs, hs)
    assert calls[0] == ("wait", "aux", "hs")
    assert [c[0] for c in calls[1:4]] == ["wide"] * 3
    assert [c[3] for c in calls[1:4]] == ["hs", "aux", "hs"]  # alternating
    assert [c[2] for c in calls[1:4]] == [400, 300, 200]      # each its own chunk
    assert calls[4] == ("wait", "hs", "aux")
    assert cost.tolist() == [400, 300, 200] and end.tolist() == [-400, -300, -200]


def test_one_chunk_stays_on_its_stream(calls):
    t = Target(4, calls)
    handles, codes, offs = _batch([400])
    Server(srv.ServerConfig(wide_streams=2))._extend(t, handles, codes, offs,
                                                      FakeStream("hs", calls))
    assert calls == [("wide", id(handles[0]), 400, "hs")]


@pytest.mark.parametrize("wide_max,lens,rows", [
    (4, [400] * 5, 0),        # more chunks than wide_max
    (0, [400], 0),            # never
    (4, [400, 400], 3800),    # a stream would pass 4,096 rows
])
def test_other_batches_take_one_launch(calls, wide_max, lens, rows):
    t = Target(wide_max, calls)
    handles, codes, offs = _batch(lens, rows)
    Server()._extend(t, handles, codes, offs, FakeStream("hs", calls))
    assert calls == [("batch", len(lens), "hs")]


def test_configured_counts_need_no_device():
    # a configured wide_chunks (>= 0) is taken as it is for int16 targets;
    # float32 targets never go over the whole device
    log = []
    s = Server(srv.ServerConfig(wide_chunks=7))
    assert s._wide_max(Target(0, log), None, None) == 7
    assert s._wide_max(Target(0, log, dtype=sd.F32), None, None) == 0
    s = Server(srv.ServerConfig(wide_chunks=-1))
    assert s._wide_max(Target(0, log, dtype=sd.F32), None, None) == 0


def test_no_room_for_the_timing_rows_means_batched_only(monkeypatch):
    # calibration opens two rows to time both paths; a budget without room
    # for them leaves the target on batched launches
    class Full:
        def __init__(self, ref):
            raise sd.SdtwError(3, "budget")  # SDTW_EBUDGET
    monkeypatch.setattr(sd, "Stream", Full)
    s = Server(srv.ServerConfig(wide_chunks=-1))
    assert s._wide_max(Target(0, []), None, None) == 0
