"""Model of the batch kernel's work pull (CPU only).

The persistent batch kernel takes reads from a longest-first list with one
64-bit atomic add on a pull word: the low half counts reads taken from the
front, the high half reads taken from the back, and the list is exhausted
once the two counts add up to its length.  When a launch of two-wave
workgroups has no more reads than workgroups, the workgroups whose first wave
runs on SIMD 2 or 3 of their CU take from the back.  This model replays the
same arithmetic under random interleavings and checks that every read is
taken exactly once, and that the placement the dispatcher uses pairs one
front and one back workgroup on every SIMD.
"""
import itertools

import numpy as np
import pytest


def pull(word, nwork, back):
    """One pull: the old (front, back) counts and the item (nwork: none left)."""
    f, b = word
    if back:
        word[1] += 1
    else:
        word[0] += 1
    if f + b >= nwork:
        return nwork
    return nwork - 1 - b if back else f


def run(nwork, classes, rng):
    """Workgroups (back flags in `classes`) pull until the list is exhausted,
    in a random interleaving; returns the items each took."""
    word = [0, 0]
    taken = [[] for _ in classes]
    live = list(range(len(classes)))
    while live:
        g = live[int(rng.integers(len(live)))]
        it = pull(word, nwork, classes[g])
        if it >= nwork:
            live.remove(g)
        else:
            taken[g].append(it)
    return taken


@pytest.mark.parametrize("nwork,groups", [(0, 4), (1, 4), (7, 8), (8, 8), (64, 64), (100, 64),
                                          (1000, 64), (5, 64)])
def test_every_item_exactly_once(nwork, groups):
    rng = np.random.default_rng(nwork * 131 + groups)
    for trial in range(20):
        classes = [bool(c) for c in rng.integers(0, 2, size=groups)]
        if trial == 0:
            classes = [False] * groups  # front only, the many-reads case
        taken = run(nwork, classes, rng)
        flat = sorted(itertools.chain.from_iterable(taken))
        assert flat == list(range(nwork))
        # front pulls take a prefix in order, back pulls a suffix in reverse
        fronts = sorted(i for g, t in enumerate(taken) if not classes[g] for i in t)
        backs = sorted(i for g, t in enumerate(taken) if classes[g] for i in t)
        assert fronts == list(range(len(fronts)))
        assert backs == list(range(nwork - len(backs), nwork))


def test_one_read_per_workgroup_when_all_pull_first():
    # every workgroup resident at once pulls before any finishes its read
    nwork, groups = 1024, 1024
    rng = np.random.default_rng(3)
    classes = [bool(c) for c in rng.integers(0, 2, size=groups)]
    word = [0, 0]
    first = [pull(word, nwork, c) for c in classes]
    assert sorted(first) == list(range(nwork))
    # the front class holds the longest reads, the back class the shortest
    nf = classes.count(False)
    assert sorted(i for i, c in zip(first, classes) if not c) == list(range(nf))


def test_placement_pairs_front_and_back_on_every_simd():
    # SIMDs of a CU's four two-wave workgroups as the dispatcher places them:
    # first wave on s, second on 2, 3, 1, 0 for s = 0, 1, 2, 3
    pairs = [(0, 2), (1, 3), (2, 1), (3, 0)]
    for order in itertools.permutations(pairs):
        load = {s: [] for s in range(4)}
        for s0, s1 in order:
            back = s0 >= 2
            load[s0].append(back)
            load[s1].append(back)
        for s in range(4):
            assert sorted(load[s]) == [False, True], (order, s, load[s])
