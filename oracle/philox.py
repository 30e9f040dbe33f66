"""Oracle: Philox4x32-10 counter-based generator (test infrastructure only).

The paper does not fix a random-number generator (its Metropolis sampler, Sec. 2.2.5,
only needs one). Both sides of the parity tests draw every random number from
Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random numbers:
as easy as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key, ten rounds of two
32x32->64-bit multiplications with the Weyl key schedule. This module is written from
that definition; the library has its own implementation.

Stream layout used by the sampler (a convention both sides follow):
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (chain, sweep, step, tag), tag 0 = Metropolis proposal, tag 1 = chain init,
            tag 2 = replica swap of parallel tempering (step = index of the swapped pair).
  word 0  -> integer index in [0, n) as floor(w0 * n / 2**32)
  words 1,2 -> uniform u = ((w1 << 21) | (w2 >> 11)) * 2**-53 in [0, 1).

Pinned by the published known-answer vectors of the generator
(``tests/golden/philox4x32_10_kat.txt``).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

TAG_PROPOSAL = 0
TAG_INIT = 1
TAG_SWAP = 2


def philox4x32_10(ctr, key):
    """ctr: uint array [..., 4]; key: uint array [..., 2] (broadcastable).
    Returns uint32 array [..., 4]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK32 for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c[0]          # exact: both factors < 2**32
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def key_from_seed(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64)


def draw(seed, chain, sweep, step, tag):
    """Philox words for arrays of (chain, sweep, step, tag) counters -> uint32 [..., 4]."""
    chain, sweep, step, tag = np.broadcast_arrays(
        np.asarray(chain, dtype=np.uint64), np.asarray(sweep, dtype=np.uint64),
        np.asarray(step, dtype=np.uint64), np.asarray(tag, dtype=np.uint64))
    ctr = np.stack([chain, sweep, step, tag], axis=-1)
    return philox4x32_10(ctr, key_from_seed(seed))


def index_from_word(w0, n):
    """floor(w0 * n / 2**32): an integer in [0, n)."""
    return ((np.asarray(w0, dtype=np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def uniform_from_words(w1, w2):
    """53-bit uniform in [0, 1) from two 32-bit words."""
    hi = np.asarray(w1, dtype=np.uint64) << np.uint64(21)
    lo = np.asarray(w2, dtype=np.uint64) >> np.uint64(11)
    return (hi | lo).astype(np.float64) * 2.0 ** -53
