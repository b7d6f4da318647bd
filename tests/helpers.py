"""Checkers shared by the tests: the plain definition of the sort result.

The expected output of every sort is the unique non-decreasing permutation of
the input under totalOrder (f64) or unsigned order (u64).  These helpers state
that definition with numpy library routines; they share nothing with either
the oracle or the GPU library.
"""
import numpy as np

SIGN = np.uint64(1 << 63)


def ord_words(a: np.ndarray) -> np.ndarray:
    """u64 words whose unsigned order is totalOrder of the f64 keys."""
    if a.dtype == np.uint64:
        return a
    w = np.ascontiguousarray(a).view(np.uint64)
    return np.where(w & SIGN, ~w, w | SIGN)


def expected_sorted(a: np.ndarray) -> np.ndarray:
    """Reference result as raw words (f64 bits or u64)."""
    o = np.sort(ord_words(a))
    if a.dtype == np.uint64:
        return o
    return np.where(o & SIGN, o & ~SIGN, ~o)


def raw_words(a: np.ndarray) -> np.ndarray:
    return a if a.dtype == np.uint64 else np.ascontiguousarray(a).view(np.uint64)


def mix64(x: np.ndarray) -> np.ndarray:
    """A 64-bit bijective mixer (fingerprints; not the sampler)."""
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xFF51AFD7ED558CCD)
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xC4CEB9FE1A85EC53)
        x ^= x >> np.uint64(33)
    return x


def fingerprint(words: np.ndarray) -> tuple:
    """(count, sum of mix64 mod 2^64, xor of mix64): equal for permutations."""
    m = mix64(words)
    with np.errstate(over="ignore"):
        s = np.add.reduce(m, dtype=np.uint64) if m.size else np.uint64(0)
    x = np.bitwise_xor.reduce(m) if m.size else np.uint64(0)
    return (int(words.size), int(s), int(x))


SPECIAL_F64 = np.array([-np.inf, -1.5, -0.0, 0.0, 5e-324, 1.0, 2.0 ** 53, np.inf])


def fingerprint_chunked(words: np.ndarray, chunk: int = 1 << 25) -> tuple:
    """fingerprint() of a large array, computed piece by piece."""
    s, x = 0, 0
    for lo in range(0, words.size, chunk):
        _, ps, px = fingerprint(words[lo:lo + chunk])
        s = (s + ps) & ((1 << 64) - 1)
        x ^= px
    return (int(words.size), s, x)


def is_sorted_words(o: np.ndarray, chunk: int = 1 << 26) -> bool:
    """Adjacent order words non-decreasing, checked piece by piece."""
    for lo in range(0, max(o.size - 1, 0), chunk):
        hi = min(o.size, lo + chunk + 1)
        if not np.all(o[lo + 1:hi] >= o[lo:hi - 1]):
            return False
    return True
