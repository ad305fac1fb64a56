"""Definition-level checks for tiny sDTW problems.  TEST INFRASTRUCTURE ONLY.

``enumerate_paths`` walks every warping path explicitly, with no memoisation,
so it evaluates the sDTW problem statement of section 2.3 directly: align all
of X (length M) with any contiguous stretch of Y (length N) using the three
step kinds of Eq. 1 (insertion (1,0), match (1,1), deletion (0,1)), and sum
the per-sample Manhattan distances along the path.  The end position is the
column of the path's last cell, and among optimal paths the smallest end
column is reported (the strict-less scan of the last row in Algorithms 1/2).

``full_matrix`` fills the whole M x N matrix of Eq. 1 with its boundary
conditions, the textbook O(MN)-space form of Algorithm 1 (section 2.3), using
exact Python integers or fractions.

Both are pure Python and meant for M, N of a handful of samples.
"""
from __future__ import annotations

INF = float("inf")


def enumerate_paths(x, y):
    """Return (cost, end0) by exhaustive enumeration of all warping paths.

    end0 is the 0-based column of the last path cell (paper's j minus 1).
    Values may be ints, Fractions or floats; sums are exact for ints/Fractions.
    """
    M, N = len(x), len(y)
    if M < 1 or N < 1:
        raise ValueError("need M >= 1 and N >= 1")
    best = {}  # end column -> minimum total cost over paths ending there

    def walk(i, j, acc):
        # the path currently ends at cell (i, j) (0-based) with total acc
        if i == M - 1:
            if j not in best or acc < best[j]:
                best[j] = acc
        # every successor of a path cell; a path may continue after reaching
        # the last row only by deletions (0,1), which stay in that row
        if i + 1 < M:
            walk(i + 1, j, acc + abs(x[i + 1] - y[j]))          # insertion
            if j + 1 < N:
                walk(i + 1, j + 1, acc + abs(x[i + 1] - y[j + 1]))  # match
        if j + 1 < N:
            walk(i, j + 1, acc + abs(x[i] - y[j + 1]))          # deletion

    for j0 in range(N):  # free start: the first path cell is (0, j0)
        walk(0, j0, abs(x[0] - y[j0]))
    cost = min(best.values())
    end0 = min(j for j, c in best.items() if c == cost)
    return cost, end0


def full_matrix(x, y):
    """Fill gamma[0..M][0..N] of Eq. 1 with its boundaries; return (gamma, cost, end0).

    gamma[0][j] = 0 for j >= 1, gamma[i][0] = inf for i >= 1 (gamma[0][0] is
    set to 0; it never decides a minimum because gamma[0][1] = 0).
    """
    M, N = len(x), len(y)
    if M < 1 or N < 1:
        raise ValueError("need M >= 1 and N >= 1")
    g = [[0] * (N + 1) for _ in range(M + 1)]
    for i in range(1, M + 1):
        g[i][0] = INF
    for i in range(1, M + 1):
        for j in range(1, N + 1):
            g[i][j] = abs(x[i - 1] - y[j - 1]) + min(g[i - 1][j], g[i - 1][j - 1],
                                                     g[i][j - 1])
    last = g[M][1:]
    cost = min(last)
    end0 = last.index(cost)
    return g, cost, end0
