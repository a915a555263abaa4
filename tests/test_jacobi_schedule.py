"""Host-side checks of the pair order of the one-sided Jacobi SVD (svd(B) of Alg. 4, steps 16-19),
through the library's own schedule generator (the code the kernel runs), without a GPU."""
import numpy as np
import pytest

import paper_1704_07669_amd as sk


def _rounds(n):
    r = 0
    while n > 1:
        h = (n + 1) // 2
        r += h
        n = h
    return r


@pytest.mark.parametrize("n", list(range(0, 129)))
def test_every_pair_once_per_sweep(n):
    tab, rounds = sk.sketch_jacobi_schedule(n)
    N = n + (n % 2)
    assert rounds == _rounds(N)
    t = np.frombuffer(tab, dtype=np.uint8).reshape(rounds, 64, 2)
    seen = np.zeros((max(N, 1), max(N, 1)), dtype=np.int64)
    for r in range(rounds):
        home, vis = t[r, :, 0].astype(int), t[r, :, 1].astype(int)
        idle = home == 255
        assert np.array_equal(idle, vis == 255)
        cols = np.concatenate([home[~idle], vis[~idle]])
        assert len(set(cols.tolist())) == len(cols)          # disjoint pairs within a round
        assert cols.size == 0 or cols.max() < N
        for p, q in zip(home[~idle], vis[~idle]):
            seen[min(p, q), max(p, q)] += 1
    iu = np.triu_indices(N, 1) if N > 1 else (np.array([], int), np.array([], int))
    assert np.all(seen[iu] == 1)                              # each pair exactly once
    assert seen.sum() == N * (N - 1) // 2


def test_homes_stay_with_their_groups():
    # a group changes its home only where a level ends: at most one change per group per level
    tab, rounds = sk.sketch_jacobi_schedule(100)
    t = np.frombuffer(tab, dtype=np.uint8).reshape(rounds, 64, 2)
    changes = 0
    for g in range(64):
        prev = None
        for r in range(rounds):
            h = int(t[r, g, 0])
            if h != 255 and h != prev:
                changes += 1
            prev = h if h != 255 else None
    assert rounds == 102
    assert changes <= 64 * 7
    assert changes < 4950 // 10


def test_bad_sizes_are_rejected():
    for n in (-1, 129):
        with pytest.raises(sk.SketchError):
            sk.sketch_jacobi_schedule(n)
