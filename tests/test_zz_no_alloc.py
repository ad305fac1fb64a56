"""sdtw_align_one_wide_noalloc, called through the C ABI, against the entry
point that owns its scratch (sdtw_align_one_wide): bit-exact cost and end on
two calls in a row, the second on a smaller input, and the size limit of the
fixed scratch array rejected before any launch."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2211_07340_amd")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(lib, ref, q, cost, end, cols=0):
    p = C.c_void_p
    return lib.sdtw_align_one_wide_noalloc(ref.handle, p(q.data_ptr()), q.numel(), cols,
                                           p(cost.data_ptr()), p(end.data_ptr()),
                                           p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_equals_wide_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = sd.load_library()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(61)
    cost = torch.full((1,), -7, dtype=torch.int32, device=dev)
    end = torch.full((1,), -7, dtype=torch.int32, device=dev)
    # first call: 400 rows x 300,000 columns; second: 90 rows x 59,796 columns
    for n, m, cols in ((300_000, 400, 0), (59_796, 90, 8)):
        r = rng.integers(-3000, 3000, size=n).astype(np.int16)
        qn = rng.integers(-3000, 3000, size=m).astype(np.int16)
        qn[: m // 2] = r[1000:1000 + m // 2]  # a partial exact occurrence
        ref = sd.Reference(torch.from_numpy(r).to(dev))
        q = torch.from_numpy(qn).to(dev)
        note(f"noalloc N={n} M={m} cols={cols}")
        want_c, want_e = sd.align_one_wide(ref, q, cols=cols)
        assert _noalloc(lib, ref, q, cost, end, cols) == 0, lib.sdtw_last_error()
        torch.cuda.synchronize()
        assert (int(cost.item()), int(end.item())) == (int(want_c.item()), int(want_e.item()))
        ref.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = sd.load_library()
    dev = torch.device("cuda:0")
    ref = sd.Reference(torch.zeros(300_000, dtype=torch.int16, device=dev))
    q = torch.zeros(4096, dtype=torch.int16, device=dev)
    cost = torch.full((1,), -7, dtype=torch.int32, device=dev)
    end = torch.full((1,), -7, dtype=torch.int32, device=dev)
    # 4,096 rows x 147 tiles of 8 columns per thread: 1.2 M words > 2^20
    assert _noalloc(lib, ref, q, cost, end, 8) == 1
    assert b"fixed array" in lib.sdtw_last_error()
    torch.cuda.synchronize()
    assert (int(cost.item()), int(end.item())) == (-7, -7)  # nothing written
    ref.close()
