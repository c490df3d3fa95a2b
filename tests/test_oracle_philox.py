"""Pins the oracle's Philox4x64-10 to numpy.random.Philox (an independent implementation)."""

import numpy as np
import pytest

from oracle.philox import philox4x64_10
from oracle.sampling import draw_uniform_words

M64 = (1 << 64) - 1


def _numpy_block(key, counter):
    """numpy's Philox increments its 256-bit counter before producing a block."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter)) - 1
    c &= (1 << 256) - 1
    words = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((0, 0), (1, 0, 0, 0)),
    ((12345, 678), (5, 1, 0, 0)),
    ((M64, 3), (M64, 7, 9, 11)),
    ((0xDEADBEEF, 0xC0FFEE), (2**40 + 17, 3, 399, 0)),
])
def test_philox_matches_numpy(key, counter):
    mine = [int(w) for w in philox4x64_10([np.uint64(c) for c in counter], key)]
    assert mine == _numpy_block(key, counter)


def test_philox_vectorised_counters():
    key = (7, 11)
    t = np.arange(50, dtype=np.uint64)
    out = philox4x64_10([t, np.uint64(1), np.uint64(2), np.uint64(0)], key)
    for k in (0, 1, 17, 49):
        ref = _numpy_block(key, (k, 1, 2, 0))
        assert [int(out[w][k]) for w in range(4)] == ref


def test_word_layout_per_mode():
    # mode n uses counter word 1 = n // 4 and output word n % 4; word 2 = row
    m, N = 9, 6
    words = draw_uniform_words(m, N, seed=3, stream=5, row=4)
    for t in (0, 8):
        for n in range(N):
            ref = _numpy_block((3, 5), (t, n // 4, 4, 0))[n % 4]
            assert int(words[t, n]) == ref
