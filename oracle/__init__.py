"""CPU oracle for subsequence DTW (HARU, arXiv 2211.07340).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2211_07340_amd``) never imports, links or executes anything
here, and this package imports nothing from it: the two share no code.

What it computes (each function cites the passage it follows):

* ``kmer_signal``   -- k-mer model conversion of a genome into the expected
  current for the forward and reverse-complement strands (section 2.2, k-mer
  model lookup over a sliding window; section 4.1, both strands).
* ``znorm``         -- z-score normalisation, statistics in double (section 4.1);
  ``zstats`` / ``zapply`` split it for reads that arrive in chunks.
* ``quantize``      -- fixed-point scaling to int16 (section 4.1; section 4.3,
  fixed-point data representation).
* ``sdtw_i64``, ``sdtw_f32``, ``sdtw_f64`` -- sDTW cost and end position
  (section 2.3, Eq. 1 and its boundary conditions; evaluated column by column
  with an (M+1) cost array as Algorithm 2 of section 4.3 describes).
* ``batch``         -- the same over a CSR batch of reads with POSIX threads.
* ``best_two``      -- the best end and the best end outside a window around
  it, on a last row (the two mapped positions a MAPQ-like decision compares;
  section 5.1 computes a mapping quality from the positions and scores).

* ``oracle.events`` -- event detection on raw samples (section 4.1's
  pre-processing with the two-window t-test detector whose R9.4 parameters
  section 5.2 takes from f5c and nanopolish), and prefix trimming; plain
  Python.

The C source is ``sdtw_oracle.c``; ``build()`` compiles it with gcc.  The
brute-force warping-path enumerator and the full-matrix recurrence used to pin
the C code live in ``oracle.brute``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdtw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

I64, F32, F64 = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = C.CDLL(_LIB_PATH)
    p = C.c_void_p
    i64 = C.c_int64
    lib.oracle_kmer_signal.argtypes = [p, i64, C.c_int, p, p]
    lib.oracle_kmer_signal.restype = i64
    lib.oracle_znorm.argtypes = [p, i64, p]
    lib.oracle_znorm.restype = None
    lib.oracle_zstats.argtypes = [p, i64, p]
    lib.oracle_zstats.restype = None
    lib.oracle_zapply.argtypes = [p, i64, C.c_double, C.c_double, p]
    lib.oracle_zapply.restype = None
    lib.oracle_quantize.argtypes = [p, i64, C.c_double, p]
    lib.oracle_quantize.restype = i64
    for name in ("oracle_sdtw_i64", "oracle_sdtw_f32", "oracle_sdtw_f64"):
        fn = getattr(lib, name)
        fn.argtypes = [p, i64, p, i64, p, p, p]
        fn.restype = None
    lib.oracle_batch.argtypes = [C.c_int, p, p, p, i64, p, i64, C.c_int, p, p]
    lib.oracle_batch.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def kmer_signal(genome: np.ndarray, table: np.ndarray, k: int) -> np.ndarray:
    """Forward || reverse-complement k-mer current signal, length 2(L-k+1)."""
    g = np.ascontiguousarray(genome, dtype=np.uint8)
    t = np.ascontiguousarray(table, dtype=np.float32)
    if t.size != 4 ** k:
        raise ValueError("table must have 4**k entries")
    L = g.size
    if L < k:
        raise ValueError("genome shorter than k")
    out = np.empty(2 * (L - k + 1), dtype=np.float32)
    n = _load().oracle_kmer_signal(_ptr(g), L, k, _ptr(t), _ptr(out))
    assert n == out.size
    return out


def znorm(v: np.ndarray) -> np.ndarray:
    """z-score with population sd, statistics in double, output float32."""
    a = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty_like(a)
    if a.size:
        _load().oracle_znorm(_ptr(a), a.size, _ptr(out))
    return out


def zstats(v: np.ndarray):
    """(mean, population sd) of v, accumulated in double in index order."""
    a = np.ascontiguousarray(v, dtype=np.float32)
    out = np.zeros(2, np.float64)
    _load().oracle_zstats(_ptr(a), a.size, _ptr(out))
    return float(out[0]), float(out[1])


def zapply(v: np.ndarray, mean: float, sd: float) -> np.ndarray:
    """(v - mean) / sd in double, rounded to float32 (zeros when sd == 0)."""
    a = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty_like(a)
    if a.size:
        _load().oracle_zapply(_ptr(a), a.size, float(mean), float(sd), _ptr(out))
    return out


def quantize(z: np.ndarray, scale: float = 64.0):
    """int16 codes = saturate(round_half_even(z * scale)); returns (codes, nsat)."""
    a = np.ascontiguousarray(z, dtype=np.float32)
    out = np.empty(a.size, dtype=np.int16)
    nsat = _load().oracle_quantize(_ptr(a), a.size, float(scale), _ptr(out))
    return out, int(nsat)


def _check_mn(x, y):
    if x.size < 1 or y.size < 1:
        raise ValueError("sDTW needs M >= 1 and N >= 1")


def sdtw_i64(x: np.ndarray, y: np.ndarray, lastrow: bool = False):
    """Exact integer sDTW on int16 inputs: (cost:int, end:int[, lastrow int64[N]])."""
    x = np.ascontiguousarray(x, dtype=np.int16)
    y = np.ascontiguousarray(y, dtype=np.int16)
    _check_mn(x, y)
    c = np.zeros(1, np.int64)
    e = np.zeros(1, np.int64)
    lr = np.empty(y.size, np.int64) if lastrow else None
    _load().oracle_sdtw_i64(_ptr(x), x.size, _ptr(y), y.size, _ptr(c), _ptr(e),
                            _ptr(lr) if lastrow else None)
    return (int(c[0]), int(e[0]), lr) if lastrow else (int(c[0]), int(e[0]))


def sdtw_f32(x: np.ndarray, y: np.ndarray, lastrow: bool = False):
    """float32-sequenced sDTW: (cost:np.float32, end:int[, lastrow float32[N]])."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    _check_mn(x, y)
    c = np.zeros(1, np.float32)
    e = np.zeros(1, np.int64)
    lr = np.empty(y.size, np.float32) if lastrow else None
    _load().oracle_sdtw_f32(_ptr(x), x.size, _ptr(y), y.size, _ptr(c), _ptr(e),
                            _ptr(lr) if lastrow else None)
    return (c[0], int(e[0]), lr) if lastrow else (c[0], int(e[0]))


def sdtw_f64(x: np.ndarray, y: np.ndarray, lastrow: bool = False):
    """double sDTW on float32 inputs: (cost:float, end:int[, lastrow float64[N]])."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    _check_mn(x, y)
    c = np.zeros(1, np.float64)
    e = np.zeros(1, np.int64)
    lr = np.empty(y.size, np.float64) if lastrow else None
    _load().oracle_sdtw_f64(_ptr(x), x.size, _ptr(y), y.size, _ptr(c), _ptr(e),
                            _ptr(lr) if lastrow else None)
    return (float(c[0]), int(e[0]), lr) if lastrow else (float(c[0]), int(e[0]))


def batch(kind: int, q: np.ndarray, offsets: np.ndarray, ref: np.ndarray,
          index=None, nthreads: int | None = None):
    """Run sDTW ``kind`` (I64/F32/F64) over CSR reads; returns (cost f64[], end i64[], threads).

    ``index`` optionally selects a subset of reads (results follow its order).
    """
    if kind == I64:
        q = np.ascontiguousarray(q, dtype=np.int16)
        ref = np.ascontiguousarray(ref, dtype=np.int16)
    else:
        q = np.ascontiguousarray(q, dtype=np.float32)
        ref = np.ascontiguousarray(ref, dtype=np.float32)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    nq = offs.size - 1
    if np.any(np.diff(offs) < 1) or ref.size < 1:
        raise ValueError("every read needs M >= 1 and the reference N >= 1")
    idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
    nrun = nq if idx is None else idx.size
    cost = np.empty(nrun, np.float64)
    end = np.empty(nrun, np.int64)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    used = _load().oracle_batch(kind, _ptr(q), _ptr(offs),
                                None if idx is None else _ptr(idx), nrun,
                                _ptr(ref), ref.size, int(nthreads),
                                _ptr(cost), _ptr(end))
    return cost, end, int(used)


def prepare_reference(genome: np.ndarray, table: np.ndarray, k: int,
                      scale: float = 64.0):
    """Section 4.1 reference preparation: k-mer signal of both strands, joint
    z-score over the concatenation, int16 codes at ``scale``.
    Returns (z float32[N], codes int16[N], nsat)."""
    sig = kmer_signal(genome, table, k)
    z = znorm(sig)
    codes, nsat = quantize(z, scale)
    return z, codes, nsat


def prepare_queries(values: np.ndarray, offsets: np.ndarray, scale: float = 64.0):
    """Section 4.1 query preparation: each read z-scored with its own
    statistics, then int16 codes at the reference's scale.
    Returns (z float32[], codes int16[], nsat)."""
    offs = np.asarray(offsets, dtype=np.int64)
    v = np.ascontiguousarray(values, dtype=np.float32)
    z = np.empty_like(v)
    for r in range(offs.size - 1):
        a, b = int(offs[r]), int(offs[r + 1])
        z[a:b] = znorm(v[a:b])
    codes, nsat = quantize(z, scale)
    return z, codes, nsat


def best_two(row: np.ndarray, window: int):
    """Best and runner-up ends of a last row gamma(M, .) (0-based columns).

    best = the first j with the minimum value (the strict-less scan of
    Algorithms 1 and 2); second = the first j with the minimum value among
    the columns with |j - best| > window.  Returns (best value, best j,
    second value, second j); second is (inf, -1) when no column lies outside
    the window.  Values are compared as given (int64 or float).
    """
    row = np.asarray(row)
    if row.size == 0 or window < 0:
        raise ValueError("empty row or negative window")
    jb = int(np.argmin(row))  # numpy returns the first index of the minimum
    j = np.arange(row.size)
    out = np.abs(j - jb) > window
    if not out.any():
        return row[jb], jb, float("inf"), -1
    # among the outside columns only: the first index attaining their minimum
    m = row[out].min()
    js = int(np.nonzero(out & (row == m))[0][0])
    return row[jb], jb, m, js
