"""Uniform 32-bit integers J for the path generators.

The paper only says that the full-precision uniform is a D-bit integer J and the
low-precision one a d-bit integer j (Section 3, notation paragraph before 3.1).
It names no generator.  Reading R1: J comes from Philox4x32-10 (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), D = 32.

Counter layout (reading R1, "global stream" form).  For one
(seed, option, level l, estimator) the uniforms form one stream of 32-bit words.
Path i, fine step n (0 <= n < 2^l) takes stream position g = i * 2^l + n.

* Unpacked (one word per step): word index w = g.
* Packed (approximate-only estimator, F = floor(32/q) table indices per word):
  word index w = g div F, field j = g mod F = bits [32-q(j+1), 32-qj) of the word.
  Field 0 is the top q bits, i.e. the same index the unpacked form uses.

Philox block b = w div 4, word w mod 4 of its output.  Counter
(c0, c1, c2, c3) = (b mod 2^32, b div 2^32, l | estimator << 8, option),
key (k0, k1) = (seed mod 2^32, seed div 2^32).

This module is test infrastructure: see the package docstring.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 block function (Salmon et al. 2011, the Philox-4x32 S-box
    with 10 rounds).  Arguments are arrays (or scalars) of uint32 values; the
    key is bumped by the Weyl constants (W0, W1) between rounds.

    One round:  (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2  (32x32 -> 64 bit),
                c <- (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0).
    Returns four uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(MASK32)
                      for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & np.uint64(MASK32)
    k1 = np.asarray(k1, dtype=np.uint64) & np.uint64(MASK32)
    m0, m1, m = np.uint64(M0), np.uint64(M1), np.uint64(MASK32)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
        p0 = m0 * c0              # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & m
        hi1, lo1 = p1 >> s32, p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def stream_counter_hi(level, estimator):
    """c2 of the counter: level in bits 0-7, estimator id in bits 8-15 (R1)."""
    return (int(level) & 0xFF) | ((int(estimator) & 0xFF) << 8)


def stream_words(seed, option, level, estimator, word_index):
    """32-bit words at the given stream word indices (uint64 array) of the
    stream (seed, option, level, estimator)."""
    w = np.asarray(word_index, dtype=np.uint64)
    b = w >> np.uint64(2)
    sel = (w & np.uint64(3)).astype(np.int64)
    c0 = b & np.uint64(MASK32)
    c1 = b >> np.uint64(32)
    c2 = np.full_like(b, stream_counter_hi(level, estimator))
    c3 = np.full_like(b, int(option) & MASK32)
    seed = int(seed)
    out = philox4x32_10(c0, c1, c2, c3, seed & MASK32, (seed >> 32) & MASK32)
    stacked = np.stack(out, axis=0)
    return stacked[sel, np.arange(w.size)].reshape(w.shape)


class StepWords:
    """The word J (unpacked) used by each path of a set at fine step n.

    Recomputes Philox for every request: slow and obviously in step with the
    layout above."""

    def __init__(self, seed, option, level, estimator, paths):
        self.seed, self.option = int(seed), int(option)
        self.level, self.est = int(level), int(estimator)
        self.paths = np.asarray(paths, dtype=np.uint64)

    def word(self, n):
        if self.level < 2:
            g = self.paths * np.uint64(1 << self.level) + np.uint64(n)
            return stream_words(self.seed, self.option, self.level, self.est, g)
        # level >= 2: a path's four steps 4m..4m+3 are the four words of one block
        if n % 4 == 0 or getattr(self, "_block_n", None) != n - n % 4:
            g0 = self.paths * np.uint64(1 << self.level) + np.uint64(n - n % 4)
            b = g0 >> np.uint64(2)
            self._words = philox4x32_10(b & np.uint64(MASK32), b >> np.uint64(32),
                                        stream_counter_hi(self.level, self.est),
                                        self.option & MASK32,
                                        self.seed & MASK32, (self.seed >> 32) & MASK32)
            self._block_n = n - n % 4
        return self._words[n % 4]

    def packed_index(self, n, q):
        """Table index of fine step n in the packed form (F = 32 // q fields
        per word, field 0 = top q bits)."""
        F = 32 // q
        g = self.paths * np.uint64(1 << self.level) + np.uint64(n)
        w = g // np.uint64(F)
        j = (g % np.uint64(F)).astype(np.int64)
        J = stream_words(self.seed, self.option, self.level, self.est, w).astype(np.int64)
        shift = 32 - q * (j + 1)
        return (J >> shift) & ((1 << q) - 1)
