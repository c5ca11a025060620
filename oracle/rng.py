"""Counter-based random numbers that fix an estimator's draws for a seed.

The paper leaves the random source unspecified (Sec. 5.1 draws pivots
uniformly, Sec. 5.2 draws a random projection Q).  The reading used here:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the output
  function z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
  z *= 0x94D049BB133111EB; z ^= z>>31.
* A keyed counter hash H(seed, tag, a, b) = s(s(s(seed ^ tag) ^ a) ^ b),
  where s(x) is the SplitMix64 output for state x (one step).
* Bounded integers in [0, bound) by Lemire's multiply-shift with rejection
  ("Fast random integer generation in an interval", ACM TOMACS 2019).
* Uniform k-subsets of {0..n-1} by Floyd's algorithm (Bentley and Floyd,
  "A sample of brilliance", CACM 1987).

Pure Python integers (and numpy uint64 for the vectorised sign words).
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB

TAG_JL = 0x4A4C
TAG_SAMPLE = 0x5350
TAG_SHARED = 0x5348
TAG_PAIRS = 0x4346


def splitmix_out(state: int) -> int:
    """SplitMix64 output for a state that has already been advanced."""
    z = state & MASK
    z = ((z ^ (z >> 30)) * C1) & MASK
    z = ((z ^ (z >> 27)) * C2) & MASK
    return z ^ (z >> 31)


def step(x: int) -> int:
    """One SplitMix64 step from state x: advance by GAMMA, return output."""
    return splitmix_out((x + GAMMA) & MASK)


class SplitMix64:
    """The sequential generator (used only to pin ``step`` to the published one)."""

    def __init__(self, seed: int):
        self.x = seed & MASK

    def next(self) -> int:
        self.x = (self.x + GAMMA) & MASK
        return splitmix_out(self.x)


def hash4(seed: int, tag: int, a: int, b: int) -> int:
    return step(step(step((seed ^ tag) & MASK) ^ (a & MASK)) ^ (b & MASK))


def lemire_bounded(words, bound: int) -> int:
    """Uniform integer in [0, bound) from an iterator of 64-bit words."""
    assert bound > 0
    x = next(words)
    m = x * bound
    low = m & MASK
    if low < bound:
        t = ((1 << 64) - bound) % bound
        while low < t:
            x = next(words)
            m = x * bound
            low = m & MASK
    return m >> 64


def stream(seed: int, tag: int, a: int):
    """64-bit words H(seed, tag, a, c) for c = 0, 1, 2, ..."""
    c = 0
    while True:
        yield hash4(seed, tag, a, c)
        c += 1


def sample_stream(seed: int, node: int):
    """64-bit words H(seed, TAG_SAMPLE, node, c) for c = 0, 1, 2, ..."""
    return stream(seed, TAG_SAMPLE, node)


def floyd_subset(n: int, k: int, words) -> list:
    """Uniform k-subset of {0, ..., n-1} (sorted), Floyd's algorithm."""
    k = min(k, n)
    chosen = set()
    for j in range(n - k, n):
        t = lemire_bounded(words, j + 1)
        chosen.add(j if t in chosen else t)
    return sorted(chosen)


def pivots(seed: int, node: int, n: int, k: int) -> list:
    """The pivot set S of Sec. 5.1 for query node ``node``: a uniform k-subset
    of all of V (the node itself may be drawn, as in the proof of Prop. 1)."""
    return floyd_subset(n, k, sample_stream(seed, node))


def shared_pivots(seed: int, n: int, k: int) -> list:
    """One pivot set for every query node (the literal reading of Sec. 5.1,
    where a single sample of k nodes is drawn): a uniform k-subset of V from
    the words H(seed, TAG_SHARED, 0, c)."""
    return floyd_subset(n, k, stream(seed, TAG_SHARED, 0))


def random_pairs(seed: int, n: int, count: int):
    """``count`` source/sink pairs, each uniform over the ordered pairs (s, t)
    with s != t: pair i takes s = bounded(n), b = bounded(n - 1) from the words
    H(seed, TAG_PAIRS, i, c) and t = b + (b >= s).  Returns int64 arrays."""
    assert n >= 2
    s = np.empty(count, np.int64)
    t = np.empty(count, np.int64)
    for i in range(count):
        words = stream(seed, TAG_PAIRS, i)
        a = lemire_bounded(words, n)
        b = lemire_bounded(words, n - 1)
        s[i] = a
        t[i] = b + (1 if b >= a else 0)
    return s, t


# ---- projection signs, vectorised over edges -------------------------------

def _np_step(x):
    x = x + np.uint64(GAMMA)
    x = (x ^ (x >> np.uint64(30))) * np.uint64(C1)
    x = (x ^ (x >> np.uint64(27))) * np.uint64(C2)
    return x ^ (x >> np.uint64(31))


def jl_sign_word(seed: int, word: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """64 sign bits for projection rows 64*word .. 64*word+63 of every edge
    {lo < hi}: H(seed, TAG_JL, word, lo * 2^32 + hi)."""
    with np.errstate(over="ignore"):
        h0 = _np_step(np.uint64((seed ^ TAG_JL) & MASK))
        h1 = _np_step(h0 ^ np.uint64(word & MASK))
        key = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
        return _np_step(np.full(lo.shape, h1, np.uint64) ^ key)


def jl_signs(seed: int, k: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """int8[k, m] matrix of +-1: entry (i, e) is +1 iff bit (i mod 64) of the
    sign word (seed, i div 64, edge e) is 0."""
    m = lo.shape[0]
    out = np.empty((k, m), np.int8)
    for wi in range((k + 63) // 64):
        wd = jl_sign_word(seed, wi, lo, hi)
        for b in range(min(64, k - 64 * wi)):
            bit = (wd >> np.uint64(b)) & np.uint64(1)
            out[64 * wi + b] = 1 - 2 * bit.astype(np.int8)
    return out
