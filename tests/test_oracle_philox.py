"""Pin of the oracle's Philox4x32-10 against the generator's published known answers."""
import os

import numpy as np

from oracle import philox

KAT = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_known_answers():
    n = 0
    for line in open(KAT):
        if not line.strip() or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        out = philox.philox4x32_10(np.array(v[:4], dtype=np.uint64), np.array(v[4:6], dtype=np.uint64))
        assert [int(x) for x in out] == v[6:10]
        n += 1
    assert n == 3


def test_index_and_uniform_ranges():
    w = philox.draw(7, np.arange(4096), 3, 5, 0)
    idx = philox.index_from_word(w[:, 0], 10)
    assert idx.min() >= 0 and idx.max() <= 9
    assert set(np.unique(idx)) == set(range(10))
    u = philox.uniform_from_words(w[:, 1], w[:, 2])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02
    # extremes of the word -> value maps
    assert philox.index_from_word(np.uint32(0xFFFFFFFF), 10) == 9
    assert philox.uniform_from_words(np.uint32(0xFFFFFFFF), np.uint32(0xFFFFFFFF)) == 1.0 - 2.0 ** -53
