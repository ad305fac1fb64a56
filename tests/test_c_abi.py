"""A plain C program (tests/c_abi/abi_check.c), built with gcc against
include/sdtw.h and libsdtw.so alone, drives the library without Python in
between: reference load, plan, autotune, batch alignment and a two-chunk
stream.  Its results must equal the oracle's bit for bit (int16 path).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2211_07340_amd")
SRC = os.path.join(ROOT, "tests", "c_abi", "abi_check.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libsdtw.so")):
        import __graft_entry__
        __graft_entry__.build()
    out = str(tmp_path_factory.mktemp("c_abi") / "abi_check")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-o", out, "-L", PKG, "-lsdtw", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{PKG}:{os.path.join(ROCM, 'lib')}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def test_c_client_builds_and_links(exe):
    r = subprocess.run([exe, "--version"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"


@pytest.mark.gpu
def test_c_client_matches_oracle(exe, tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    table = synth.make_level_table()
    genome = synth.make_genome(synth.SMALL_GENOME, 17)
    # ragged lengths: one event, a partial wave, full and part tiles, the cap
    lengths = np.array([1000, 1, 7, 64, 65, 250, 333, 4096] + [250] * 24 + [500] * 8)
    rd = synth.simulate_reads(genome, table, lengths, 0.5, 23)
    _, ref, _ = oracle.prepare_reference(genome, table, synth.K)
    _, q, _ = oracle.prepare_queries(rd.values, rd.offsets)
    ref.astype(np.int16).tofile(tmp_path / "ref.i16")
    q.astype(np.int16).tofile(tmp_path / "q.i16")
    offs = np.asarray(rd.offsets, np.int64)
    offs.tofile(tmp_path / "offs.i64")

    raw = synth.simulate_raw(genome, table, 5, 320, 0.6, 29)
    raw.values.tofile(tmp_path / "raw.f32")
    raw.offsets.astype(np.int64).tofile(tmp_path / "raw_offs.i64")

    print(f"abi_check {tmp_path} nq={offs.size - 1} n={ref.size}", flush=True)
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr

    nq = offs.size - 1
    got = np.fromfile(tmp_path / "batch.i32", np.int32)
    want_c, want_e, _ = oracle.batch(oracle.I64, q, offs, ref)
    np.testing.assert_array_equal(got[:nq], want_c.astype(np.int64))
    np.testing.assert_array_equal(got[nq:], want_e)

    # the stream over read 0 after its first third, then after all of it
    m0 = int(offs[1] - offs[0])
    cut = max(m0 // 3, 1)
    pre = np.array([0, cut, cut + m0], np.int64)
    qq = np.concatenate([q[:cut], q[:m0]])
    sc, se, _ = oracle.batch(oracle.I64, qq, pre, ref)
    got = np.fromfile(tmp_path / "stream.i32", np.int32)
    assert got.tolist() == [int(sc[0]), int(se[0]), int(sc[1]), int(se[1])]
    # read 0 over the whole device
    assert np.fromfile(tmp_path / "wide.i32", np.int32).tolist() == [int(sc[1]), int(se[1])]
    # event detection
    from oracle import events as oev
    ev = np.fromfile(tmp_path / "events.f32", np.float32).reshape(5, 250)
    cnt = np.fromfile(tmp_path / "event_counts.i32", np.int32)
    for r in range(5):
        want = oev.query_events(raw.values[raw.offsets[r]:raw.offsets[r + 1]], 50, 250)
        assert cnt[r] == want.size and np.array_equal(ev[r, :cnt[r]], want), r
