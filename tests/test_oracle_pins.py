"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
a hand-worked fixture (tests/golden), an exhaustive enumeration of warping
paths, a closed form, a library routine, or an invariant of the problem.
The mutation tests at the end plant plausible mistakes in Python copies of
the oracle's recurrence and check that the same pins reject each of them.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import brute
from tests.golden import load as golden

# ----------------------------------------------------------------------------
# hand-worked sDTW fixtures (section 2.3 Eq. 1)
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("case", golden.sdtw_cases(), ids=lambda c: c["NAME"])
def test_golden_sdtw(case):
    x, y = case["X"], case["Y"]
    g, cost, end0 = brute.full_matrix(x, y)
    for i, row in enumerate(case["ROWS"], start=1):
        assert g[i][1:] == row, f"gamma row {i}"
    assert (cost, end0) == (case["COST"], case["END0"])
    assert brute.enumerate_paths(x, y) == (case["COST"], case["END0"])
    xi, yi = np.array(x, np.int16), np.array(y, np.int16)
    c, e, lr = oracle.sdtw_i64(xi, yi, lastrow=True)
    assert (c, e) == (case["COST"], case["END0"])
    assert lr.tolist() == case["ROWS"][-1]
    for fn in (oracle.sdtw_f32, oracle.sdtw_f64):
        c, e, lr = fn(xi.astype(np.float32), yi.astype(np.float32), lastrow=True)
        assert (float(c), e) == (case["COST"], case["END0"])
        assert lr.tolist() == case["ROWS"][-1]


# ----------------------------------------------------------------------------
# exhaustive enumeration of warping paths (problem statement of section 2.3)
# ----------------------------------------------------------------------------


def _random_small(rng, mmax=5, nmax=5, lo=-5, hi=5):
    M = int(rng.integers(1, mmax + 1))
    N = int(rng.integers(1, nmax + 1))
    x = rng.integers(lo, hi + 1, size=M)
    y = rng.integers(lo, hi + 1, size=N)
    return x, y


def test_brute_force_all_variants():
    rng = np.random.default_rng(7)
    for _ in range(400):
        x, y = _random_small(rng)
        want = brute.enumerate_paths(x.tolist(), y.tolist())
        assert oracle.sdtw_i64(x, y) == want
        c, e = oracle.sdtw_f32(x.astype(np.float32), y.astype(np.float32))
        assert (float(c), e) == want
        c, e = oracle.sdtw_f64(x.astype(np.float32), y.astype(np.float32))
        assert (c, e) == want


def test_brute_force_six_by_six_and_ties():
    rng = np.random.default_rng(11)
    for _ in range(25):
        x = rng.integers(-1, 2, size=6)  # few distinct values: many ties
        y = rng.integers(-1, 2, size=6)
        want = brute.enumerate_paths(x.tolist(), y.tolist())
        assert oracle.sdtw_i64(x, y) == want


def test_brute_force_fractions_vs_f64():
    # dyadic fractions: every partial sum is exact in double, so the double
    # oracle must reproduce exact rational enumeration
    rng = np.random.default_rng(3)
    for _ in range(150):
        x, y = _random_small(rng, lo=-40, hi=40)
        xf = [Fraction(int(v), 8) for v in x]
        yf = [Fraction(int(v), 8) for v in y]
        want_c, want_e = brute.enumerate_paths(xf, yf)
        c, e = oracle.sdtw_f64((x / 8).astype(np.float32), (y / 8).astype(np.float32))
        assert (Fraction(c), e) == (want_c, want_e)


def test_full_matrix_matches_enumeration_and_oracle_lastrow():
    rng = np.random.default_rng(5)
    for _ in range(200):
        x, y = _random_small(rng, mmax=6, nmax=9)
        g, cost, end0 = brute.full_matrix(x.tolist(), y.tolist())
        c, e, lr = oracle.sdtw_i64(x, y, lastrow=True)
        assert lr.tolist() == g[len(x)][1:]
        assert (c, e) == (cost, end0)


# ----------------------------------------------------------------------------
# closed forms and special cases
# ----------------------------------------------------------------------------


def test_m_equals_one_is_nearest_value_search():
    # M = 1: gamma(1,j) = |x - y_j|, so (cost, end) = (min, first argmin)
    rng = np.random.default_rng(1)
    for _ in range(50):
        y = rng.normal(size=int(rng.integers(1, 300))).astype(np.float32)
        x = rng.normal(size=1).astype(np.float32)
        d = np.abs(x[0] - y)
        c, e = oracle.sdtw_f32(x, y)
        assert c == d.min() and e == int(np.argmin(d))
        yi = rng.integers(-300, 300, size=y.size).astype(np.int16)
        xi = rng.integers(-300, 300, size=1).astype(np.int16)
        di = np.abs(xi.astype(np.int64)[0] - yi.astype(np.int64))
        assert oracle.sdtw_i64(xi, yi) == (int(di.min()), int(np.argmin(di)))


def test_n_equals_one_is_column_sum():
    rng = np.random.default_rng(2)
    for _ in range(20):
        x = rng.integers(-1000, 1000, size=int(rng.integers(1, 400))).astype(np.int16)
        y = rng.integers(-1000, 1000, size=1).astype(np.int16)
        want = int(np.abs(x.astype(np.int64) - int(y[0])).sum())
        assert oracle.sdtw_i64(x, y) == (want, 0)


def test_constant_signals():
    # q == a and r == b: cost = M |a - b|, every column ties, first wins
    for M, N, a, b in [(7, 11, 3, -2), (250, 600, 100, 100), (1, 5, 0, 9)]:
        x = np.full(M, a, np.int16)
        y = np.full(N, b, np.int16)
        assert oracle.sdtw_i64(x, y) == (M * abs(a - b), 0)
        c, e = oracle.sdtw_f32(x.astype(np.float32) / 4, y.astype(np.float32) / 4)
        assert (float(c), e) == (M * abs(a - b) / 4, 0)


def test_constant_query_any_reference():
    # q == a: the best path stays in one column; cost = M min_j |a - r_j|
    rng = np.random.default_rng(4)
    for _ in range(30):
        M = int(rng.integers(1, 40))
        y = rng.integers(-50, 50, size=int(rng.integers(1, 80))).astype(np.int16)
        a = int(rng.integers(-50, 50))
        d = np.abs(a - y.astype(np.int64))
        assert oracle.sdtw_i64(np.full(M, a, np.int16), y) == (M * int(d.min()), int(np.argmin(d)))


def test_constant_reference_any_query():
    rng = np.random.default_rng(6)
    for _ in range(30):
        x = rng.integers(-50, 50, size=int(rng.integers(1, 60))).astype(np.int16)
        b = int(rng.integers(-50, 50))
        N = int(rng.integers(1, 50))
        want = int(np.abs(x.astype(np.int64) - b).sum())
        assert oracle.sdtw_i64(x, np.full(N, b, np.int16)) == (want, 0)


def test_exact_substring_has_zero_cost():
    rng = np.random.default_rng(8)
    y = rng.normal(size=5000).astype(np.float32)  # continuous: no equal runs
    for _ in range(20):
        M = int(rng.integers(1, 300))
        a = int(rng.integers(0, y.size - M + 1))
        x = y[a:a + M].copy()
        c, e = oracle.sdtw_f32(x, y)
        assert c == 0.0 and e == a + M - 1
        c, e = oracle.sdtw_f64(x, y)
        assert c == 0.0 and e == a + M - 1
        yq = np.round(y * 64).astype(np.int16)
        c, e = oracle.sdtw_i64(yq[a:a + M], yq)
        assert c == 0 and e <= a + M - 1


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------


def test_reversal_invariance():
    rng = np.random.default_rng(9)
    for _ in range(100):
        x, y = _random_small(rng, mmax=12, nmax=30, lo=-20, hi=20)
        c1, _ = oracle.sdtw_i64(x, y)
        c2, _ = oracle.sdtw_i64(x[::-1], y[::-1])
        assert c1 == c2


def test_translation_and_integer_scaling():
    rng = np.random.default_rng(10)
    for _ in range(100):
        x, y = _random_small(rng, mmax=15, nmax=40, lo=-100, hi=100)
        c, e = oracle.sdtw_i64(x, y)
        sh = int(rng.integers(-1000, 1000))
        assert oracle.sdtw_i64(x + sh, y + sh) == (c, e)
        k = int(rng.integers(2, 50))
        assert oracle.sdtw_i64(x * k, y * k) == (c * k, e)


def test_query_prefix_monotone_and_reference_prefix_local():
    rng = np.random.default_rng(12)
    for _ in range(40):
        x, y = _random_small(rng, mmax=20, nmax=60, lo=-30, hi=30)
        costs = [oracle.sdtw_i64(x[:m], y)[0] for m in range(1, x.size + 1)]
        assert all(a <= b for a, b in zip(costs, costs[1:]))
        _, _, full = oracle.sdtw_i64(x, y, lastrow=True)
        for n in range(1, y.size + 1):
            c, e, lr = oracle.sdtw_i64(x, y[:n], lastrow=True)
            # gamma(., j) depends on Y[1..j] only: the last row is a prefix
            assert np.array_equal(lr, full[:n])
            assert c == full[:n].min() and e == int(np.argmin(full[:n]))


def test_f32_close_to_f64():
    rng = np.random.default_rng(13)
    y = rng.normal(size=3000).astype(np.float32)
    for _ in range(10):
        x = rng.normal(size=250).astype(np.float32)
        c32, e32 = oracle.sdtw_f32(x, y)
        c64, e64, lr64 = oracle.sdtw_f64(x, y, lastrow=True)
        assert abs(float(c32) - c64) <= 1e-5 * c64
        assert lr64[e32] <= c64 * (1 + 1e-5)


# ----------------------------------------------------------------------------
# preparation (section 2.2 k-mer model; section 4.1 strands, z-score, scaling)
# ----------------------------------------------------------------------------


def test_kmer_golden():
    p = golden.prep_cases()
    k = int(p["KMER_K"][0])
    table = np.arange(4 ** k, dtype=np.float32)
    g = np.array(p["KMER_GENOME"], np.uint8)
    assert oracle.kmer_signal(g, table, k).tolist() == p["KMER_SIGNAL"]


def test_kmer_strand_symmetry():
    # the signal of revcomp(g) is the signal of g with its two strands swapped
    rng = np.random.default_rng(14)
    table = rng.normal(90, 12, size=4 ** 6).astype(np.float32)
    g = rng.integers(0, 4, size=500).astype(np.uint8)
    rc = (3 - g[::-1]).astype(np.uint8)
    s, t = oracle.kmer_signal(g, table, 6), oracle.kmer_signal(rc, table, 6)
    n = s.size // 2
    assert s.size == 2 * (500 - 6 + 1)
    assert np.array_equal(s[:n], t[n:]) and np.array_equal(s[n:], t[:n])
    # one-base shift moves every forward k-mer by one position
    s2 = oracle.kmer_signal(g[1:], table, 6)
    assert np.array_equal(s2[: n - 1], s[1:n])


def test_znorm_closed_form_and_library():
    p = golden.prep_cases()
    z = oracle.znorm(np.array(p["ZNORM_IN"], np.float32))
    want = (np.array(p["ZNORM_OUT_TIMES_SQRT5"]) / np.sqrt(5.0)).astype(np.float32)
    assert np.array_equal(z, want)
    rng = np.random.default_rng(15)
    for n in (1, 2, 17, 250, 4001):
        v = rng.normal(90, 12, size=n).astype(np.float32)
        z = oracle.znorm(v)
        ref = scipy.stats.zscore(v.astype(np.float64), ddof=0)
        if n == 1:
            assert z.tolist() == [0.0]
            continue
        assert np.allclose(z, ref.astype(np.float32), rtol=0, atol=4e-7 * np.abs(ref).max())
        assert abs(z.astype(np.float64).mean()) < 1e-6
        assert abs(z.astype(np.float64).std() - 1) < 1e-6
    assert oracle.znorm(np.full(10, 3.5, np.float32)).tolist() == [0.0] * 10


def test_quantize_golden():
    p = golden.prep_cases()
    z = (np.array(p["QUANT_IN_TIMES_64"]) / 64).astype(np.float32)
    codes, nsat = oracle.quantize(z, p["QUANT_SCALE"][0])
    assert codes.tolist() == [int(v) for v in p["QUANT_OUT"]]
    assert nsat == int(p["QUANT_NSAT"][0])


def test_batch_equals_single():
    rng = np.random.default_rng(16)
    ref = rng.normal(size=700).astype(np.float32)
    reads = [rng.normal(size=int(m)).astype(np.float32) for m in rng.integers(1, 90, size=23)]
    lens = np.array([r.size for r in reads])
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    q = np.concatenate(reads)
    for kind, fn, cast in [(oracle.F32, oracle.sdtw_f32, np.float32),
                           (oracle.F64, oracle.sdtw_f64, np.float32),
                           (oracle.I64, oracle.sdtw_i64, None)]:
        qq = q if cast else np.round(q * 64).astype(np.int16)
        rr = ref if cast else np.round(ref * 64).astype(np.int16)
        cost, end, used = oracle.batch(kind, qq, offs, rr, nthreads=3)
        assert used == 3
        for r in range(len(reads)):
            c, e = fn(qq[offs[r]:offs[r + 1]], rr)
            assert cost[r] == float(c) and end[r] == e
        sub = np.array([5, 2, 19])
        cost2, end2, _ = oracle.batch(kind, qq, offs, rr, index=sub, nthreads=2)
        assert np.array_equal(cost2, cost[sub]) and np.array_equal(end2, end[sub])


def test_rejects_empty():
    with pytest.raises(ValueError):
        oracle.sdtw_f32(np.zeros(0, np.float32), np.zeros(3, np.float32))
    with pytest.raises(ValueError):
        oracle.sdtw_i64(np.zeros(3, np.int16), np.zeros(0, np.int16))


# ----------------------------------------------------------------------------
# the pins reject plausible mistakes (planted in Python copies, on the CPU)
# ----------------------------------------------------------------------------


def _dp(x, y, variant):
    M, N = len(x), len(y)
    INF = float("inf")
    C = [0] + [INF] * M
    best, pos = INF, -1
    for j in range(1, N + 1):
        diag = 0
        for i in range(1, M + 1):
            up, left = C[i - 1], C[i]
            d = abs(x[i - 1] - y[j - 1])
            if variant == "drop_diag":
                m = min(up, left)
            elif variant == "drop_left":
                m = min(up, diag)
            elif variant == "no_free_start":  # gamma(0,j) = inf for j > 1
                m = min(up if (i > 1 or j == 1) else INF, diag if i > 1 else INF, left)
            elif variant == "signed_distance":
                d = x[i - 1] - y[j - 1]
                m = min(up, diag, left)
            elif variant == "transposed":  # X indexed by column, Y by row
                d = abs(x[min(j, M) - 1] - y[min(i, N) - 1])
                m = min(up, diag, left)
            elif variant == "shifted_neighbours":
                # the diagonal and left operands taken one row too low:
                # gamma(i, j-1) in place of gamma(i-1, j-1) and gamma(i+1, j-1)
                # in place of gamma(i, j-1) (the reading of Algorithm 2's
                # neighbour indices that section 2.3 Eq. 1 rules out)
                below = C[i + 1] if i < M else INF
                m = min(up, left, below)
            else:
                m = min(up, diag, left)
            C[i] = d + m
            diag = left
        cmp = (C[M] <= best) if variant == "last_tie" else (C[M] < best)
        if cmp:
            best, pos = C[M], j
    return best, pos - 1


@pytest.mark.parametrize("variant", ["drop_diag", "drop_left", "no_free_start",
                                     "signed_distance", "transposed", "last_tie",
                                     "shifted_neighbours"])
def test_pins_reject_planted_mistakes(variant):
    def fn(x, y):
        return _dp(x, y, variant)
    # the correct copy passes the same checks, so a failure below is the mistake
    rng = np.random.default_rng(21)
    cases = [_random_small(rng) for _ in range(300)]
    assert all(_dp(x.tolist(), y.tolist(), "ok") == brute.enumerate_paths(x.tolist(), y.tolist())
               for x, y in cases[:60])
    caught = any(fn(x.tolist(), y.tolist()) != brute.enumerate_paths(x.tolist(), y.tolist())
                 for x, y in cases)
    for case in golden.sdtw_cases():
        caught = caught or fn(case["X"], case["Y"]) != (case["COST"], case["END0"])
    assert caught, f"planted mistake {variant} passed every pin"


def test_shifted_neighbours_counterexample():
    # the reading recorded for the garbled neighbour indices of Algorithm 2:
    # taken one row too low they give (10, first column) on this pair, where
    # Eq. 1 gives (0, second column)
    assert _dp([0, 10], [0, 10], "shifted_neighbours") == (10, 0)
    assert brute.enumerate_paths([0, 10], [0, 10]) == (0, 1)


# ---- best and runner-up ends (decision stage) -------------------------------

def test_best_two_hand_examples():
    row = np.array([5, 1, 3, 1, 0, 2])
    assert oracle.best_two(row, 0) == (0, 4, 1, 1)   # runner-up: first of the tied 1s
    assert oracle.best_two(row, 2) == (0, 4, 1, 1)   # j in {0, 1} remain
    assert oracle.best_two(row, 3) == (0, 4, 5, 0)   # only j = 0 remains
    assert oracle.best_two(row, 4) == (0, 4, float("inf"), -1)
    # ties for the best: the first index wins, the other tie is the runner-up
    assert oracle.best_two(np.array([2, 7, 2, 9]), 1) == (2, 0, 2, 2)
    assert oracle.best_two(np.array([2, 7, 2, 9]), 2) == (2, 0, 9, 3)


def test_best_two_against_sorted_scan():
    # independent formulation: sort (value, j) lexicographically; the best is
    # the first pair, the runner-up the first later pair outside the window
    rng = np.random.default_rng(31)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        row = rng.integers(0, 6, size=n)
        w = int(rng.integers(0, 8))
        pairs = sorted((int(v), j) for j, v in enumerate(row))
        b = pairs[0]
        rest = [p for p in pairs[1:] if abs(p[1] - b[1]) > w]
        want = (b[0], b[1]) + ((rest[0][0], rest[0][1]) if rest else (float("inf"), -1))
        assert oracle.best_two(row, w) == want, (row, w)


# ---- float32 arithmetic: one rounding per subtraction and per addition -----
# (section 2.3 Eq. 1 evaluated in binary32; the fixed-point path of section
# 4.3 is pinned by the integer cases above)


def _rne32(q):
    """Round a rational to the nearest binary32 value, ties to even (IEEE 754
    round-to-nearest-even, subnormals included), exactly, as a Fraction."""
    q = Fraction(q)
    if q == 0:
        return Fraction(0)
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    quantum = Fraction(2) ** max(e - 23, -149)  # 24-bit significand; subnormal spacing
    n, rem = divmod(a / quantum, 1)
    n = int(n)
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    r = n * quantum
    assert r < Fraction(2) ** 128
    return r if q > 0 else -r


def test_rne32_matches_float32_conversion():
    # the rounding helper itself against numpy's float32 conversion
    rng = np.random.default_rng(40)
    for _ in range(2000):
        v = float(rng.normal() * 2.0 ** int(rng.integers(-140, 100)))
        assert _rne32(Fraction(v)) == Fraction(float(np.float32(v)))
    assert _rne32(Fraction(1) + Fraction(1, 2 ** 24)) == 1       # tie: to even
    assert _rne32(Fraction(1) + Fraction(3, 2 ** 24)) == 1 + Fraction(1, 2 ** 22)


def _enumerate_paths_f32(x, y):
    """Every warping path with its sum accumulated in binary32 along the path:
    acc <- rne32(|rne32(x_i - y_j)| + acc), cell by cell (exact rationals and
    explicit rounding, no hardware float).  Rounding is monotone, so
    rne32(d + min(a, b, c)) = min of rne32(d + a), rne32(d + b), rne32(d + c)
    and the recurrence of Eq. 1 in binary32 computes exactly the smallest such
    path sum at every cell: its (cost, first end) is this enumeration's."""
    M, N = len(x), len(y)
    xs = [Fraction(float(v)) for v in x]
    ys = [Fraction(float(v)) for v in y]
    best = {}

    def dist(i, j):
        return abs(_rne32(xs[i] - ys[j]))

    def walk(i, j, acc):
        if i == M - 1 and (j not in best or acc < best[j]):
            best[j] = acc
        if i + 1 < M:
            walk(i + 1, j, _rne32(dist(i + 1, j) + acc))
            if j + 1 < N:
                walk(i + 1, j + 1, _rne32(dist(i + 1, j + 1) + acc))
        if j + 1 < N:
            walk(i, j + 1, _rne32(dist(i, j + 1) + acc))

    for j0 in range(N):
        walk(0, j0, dist(0, j0))
    cost = min(best.values())
    return cost, min(j for j, c in best.items() if c == cost)


def _rounding_cases(seed, count):
    # values of mixed magnitudes, so that x - y is often not a binary32 value
    # and the additions round too
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        M, N = int(rng.integers(1, 5)), int(rng.integers(1, 6))
        x = (rng.normal(size=M) * 2.0 ** rng.integers(-12, 12, size=M)).astype(np.float32)
        y = (rng.normal(size=N) * 2.0 ** rng.integers(-12, 12, size=N)).astype(np.float32)
        out.append((x, y))
    return out


def test_f32_oracle_rounds_once_per_operation():
    rounded = 0
    for x, y in _rounding_cases(41, 300):
        want_c, want_e = _enumerate_paths_f32(x, y)
        c, e = oracle.sdtw_f32(x, y)
        assert (Fraction(float(c)), e) == (want_c, want_e), (x, y)
        rounded += any(Fraction(float(a)) - Fraction(float(b)) != _rne32(
            Fraction(float(a)) - Fraction(float(b))) for a in x for b in y)
    assert rounded > 200  # the cases exercise rounding


def _rowmajor_f32(x, y):
    """Eq. 1 filled row by row (rows outer, columns inner), keeping only the
    previous row, in numpy float32 scalars (one rounding per operation)."""
    M, N = len(x), len(y)
    inf = np.float32(np.inf)
    prev = [np.float32(0)] * N          # gamma(0, j) = 0
    for i in range(M):
        cur = []
        left, diag = inf, inf           # gamma(i, 0) = inf; gamma(i-1, 0) = inf (0 in row 1)
        if i == 0:
            diag = np.float32(0)
        for j in range(N):
            m = min(prev[j], diag, left)
            v = np.float32(abs(np.float32(x[i] - y[j])) + m)
            cur.append(v)
            diag, left = prev[j], v
        prev = cur
    c = min(prev)
    return c, prev.index(c), np.array(prev, np.float32)


def test_row_major_traversal_equals_column_major_oracle():
    # section 2.3 defines gamma cell by cell; the order in which the cells are
    # filled cannot change any of them (each is one subtraction, one min and
    # one addition of the same three operands), so a row-major pass equals
    # the column-major oracle bit for bit, last row included
    rng = np.random.default_rng(42)
    for t in range(60):
        M, N = int(rng.integers(1, 30)), int(rng.integers(1, 70))
        x = (rng.normal(size=M) * 2.0 ** rng.integers(-6, 6, size=M)).astype(np.float32)
        y = (rng.normal(size=N) * 2.0 ** rng.integers(-6, 6, size=N)).astype(np.float32)
        c, e, row = _rowmajor_f32(x, y)
        oc, oe, olr = oracle.sdtw_f32(x, y, lastrow=True)
        assert (c.tobytes(), e) == (oc.tobytes(), oe)
        assert row.tobytes() == olr.tobytes()


def _dp_f32_double_accumulate(x, y):
    """Planted mistake: each cell's distance and sum taken in double and
    rounded to binary32 once, instead of once per operation."""
    M, N = len(x), len(y)
    C = [np.float32(0)] + [np.float32(np.inf)] * M
    best, pos = np.float32(np.inf), -1
    for j in range(N):
        diag = np.float32(0)
        for i in range(1, M + 1):
            up, left = C[i - 1], C[i]
            m = min(up, diag, left)
            C[i] = np.float32(abs(float(x[i - 1]) - float(y[j])) + float(m))
            diag = left
        if C[M] < best:
            best, pos = C[M], j
    return best, pos


def test_pins_reject_double_accumulating_f32():
    caught = False
    for x, y in _rounding_cases(41, 300):
        c, e = _dp_f32_double_accumulate(x, y)
        caught = caught or (Fraction(float(c)), e) != _enumerate_paths_f32(x, y)
    assert caught


# ---- z statistics of a first chunk and their application (section 4.1) -----


def _zstats_ddof1(v):
    """Planted mistake: the sample (n - 1) variance."""
    v = np.asarray(v, np.float64)
    return float(v.mean()), float(np.sqrt(((v - v.mean()) ** 2).sum() / (v.size - 1)))


def test_zstats_hand_worked():
    p = golden.prep_cases()
    for key in ("", "2"):
        v = np.array(p["ZSTATS_IN" + key], np.float32)
        mean, sd = oracle.zstats(v)
        assert mean == p["ZSTATS_MEAN" + key][0]
        assert sd == np.sqrt(p["ZSTATS_VAR" + key][0])  # correctly rounded sqrt
        m1, s1 = _zstats_ddof1(v)
        assert s1 != sd  # the planted mistake fails this pin
    assert oracle.zstats(np.full(7, 2.5, np.float32)) == (2.5, 0.0)
    assert oracle.zstats(np.array([3.0], np.float32)) == (3.0, 0.0)


def test_zstats_against_exact_rationals():
    # mean and population sd from exact rational sums; the oracle accumulates
    # in double, so it agrees to within a few double ulps
    rng = np.random.default_rng(43)
    for n in (2, 5, 250, 2000):
        v = rng.normal(90, 12, size=n).astype(np.float32)
        fr = [Fraction(float(a)) for a in v]
        mean = sum(fr) / n
        var = sum((a - mean) ** 2 for a in fr) / n
        m, sd = oracle.zstats(v)
        assert abs(Fraction(m) - mean) <= abs(mean) * Fraction(1, 2 ** 48)
        assert abs(Fraction(sd) ** 2 - var) <= var * Fraction(1, 2 ** 46)
        _, s1 = _zstats_ddof1(v)
        assert abs(Fraction(s1) ** 2 - var) > var * Fraction(1, 2 ** 46)


def test_zapply_hand_worked_and_consistent_with_znorm():
    p = golden.prep_cases()
    mean, sd = oracle.zstats(np.array(p["ZSTATS_IN"], np.float32))
    out = oracle.zapply(np.array(p["ZAPPLY_IN"], np.float32), mean, sd)
    want = (np.array(p["ZAPPLY_OUT_TIMES_SQRT5"]) / np.sqrt(5.0)).astype(np.float32)
    assert np.array_equal(out, want)
    # sd == 0 gives zeros
    assert oracle.zapply(np.array([1, 2], np.float32), 1.0, 0.0).tolist() == [0.0, 0.0]
    # statistics of a whole read applied to that read are its z-score
    rng = np.random.default_rng(44)
    for n in (1, 3, 400, 2000):
        v = rng.normal(90, 12, size=n).astype(np.float32)
        assert oracle.zapply(v, *oracle.zstats(v)).tobytes() == oracle.znorm(v).tobytes()
