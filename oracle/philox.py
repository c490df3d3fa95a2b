"""Philox4x64-10, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11), Philox-4x64 with 10 rounds: each round multiplies counter words 0 and 2
by two fixed odd constants (full 64x64 -> 128-bit products), xors the high halves
into the other two words together with the round key, and permutes the words; the
two key words are bumped by the Weyl constants (golden ratio and sqrt(3) - 1
scaled to 64 bits) between rounds.

Pinned by tests/test_oracle_philox.py against numpy.random.Philox, an
independent implementation of the same generator.
"""

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64-bit product of uint64 arrays, as (high word, low word).

    Schoolbook product on 32-bit halves; every partial sum fits in 64 bits.
    """
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (hl & _LO32) + lh
    hi = hh + (hl >> _S32) + (cross >> _S32)
    lo = (cross << _S32) | (ll & _LO32)
    return hi, lo


def philox4x64_10(counter, key):
    """Apply Philox4x64-10 to counters.

    counter: sequence of four uint64 arrays (broadcastable), words 0..3.
    key:     two 64-bit integers.
    Returns a list of four uint64 arrays, the output words 0..3.
    """
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in counter)
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        k0 = np.uint64(int(key[0]) & 0xFFFFFFFFFFFFFFFF)
        k1 = np.uint64(int(key[1]) & 0xFFFFFFFFFFFFFFFF)
        for rnd in range(10):
            if rnd:
                k0 = np.uint64(k0 + W0)
                k1 = np.uint64(k1 + W1)
            hi0, lo0 = _mulhilo64(M0, x0)
            hi1, lo1 = _mulhilo64(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return [x0.copy(), x1.copy(), x2.copy(), x3.copy()]
