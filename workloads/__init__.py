"""Seeded synthetic inputs for the sorting workloads.

This module only draws random keys; it holds none of the sorting method's
arithmetic.  Tests and the benchmark take their inputs from here, so the GPU
path and the CPU oracle always see the same keys.

Workloads (sizes as used by the tests and the benchmark):
  uniform_1e9grid   1,000,000 f64, U[0,1) rounded down to a 1e-9 grid.
  zipf_lognormal    200,000,000 f64: Zipf(s=1.2) ranks over 100,000 distinct
                    values, each distinct value drawn lognormal(0, 2).
  mixed_u64         1,000,000,000 u64: equal thirds of round(N(2^40, 2^36)),
                    round(Exp(scale 2^30)), U[0, 2^64) mod 10,000, shuffled.
  segments          10,000 f64 arrays, sizes log-uniform in [1024, 4194304],
                    family per array: uniform, normal, lognormal, zipf-dup.
  requests          a Poisson stream of f64 / u64 sort requests, sizes
                    log-uniform in [1024, 67108864], duplicate ratio U(0, 0.99).
Paper families (Sec. 6.1 list of synthetic datasets): root_dups, two_dups,
mix_gauss, normal, lognormal(0, 0.5), chi_square(4), exponential(2),
uniform(0..N), zipf(skew).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

CHUNK = 1 << 24


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


# --------------------------------------------------------------- the configs --

def uniform_1e9grid(n: int = 1_000_000, seed: int = 1) -> np.ndarray:
    """U[0,1) doubles rounded down to multiples of 1e-9 (a few duplicates)."""
    r = _rng(seed)
    return np.floor(r.random(n) * 1e9) / 1e9


def zipf_table(distinct: int, s: float) -> np.ndarray:
    """Cumulative Zipf(s) probabilities over ranks 1..distinct."""
    w = np.arange(1, distinct + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, fill, workers: int | None = None) -> None:
    """Run fill(c, lo, hi) for every CHUNK-sized piece of [0, n), in threads
    (numpy's generators and ufuncs release the GIL on large arrays).  Each
    piece draws from its own stream, so the result does not depend on the
    number of threads."""
    pieces = [(c, lo, min(n, lo + CHUNK)) for c, lo in enumerate(range(0, n, CHUNK))]
    w = workers or _workers()
    if w == 1 or len(pieces) == 1:
        for c, lo, hi in pieces:
            fill(c, lo, hi)
        return
    with ThreadPoolExecutor(w) as ex:
        list(ex.map(lambda t: fill(*t), pieces))


def zipf_lognormal(n: int = 200_000_000, seed: int = 2, distinct: int = 100_000,
                   s: float = 1.2, sigma: float = 2.0) -> np.ndarray:
    """Zipf(s)-distributed picks among `distinct` lognormal(0, sigma) values."""
    r = _rng(seed)
    values = r.lognormal(0.0, sigma, size=distinct)
    cdf = zipf_table(distinct, s)
    out = np.empty(n, dtype=np.float64)

    def fill(c, lo, hi):
        rank = np.searchsorted(cdf, _rng(seed, 1 + c).random(hi - lo), side="right")
        np.minimum(rank, distinct - 1, out=rank)
        out[lo:hi] = values[rank]

    _chunked(n, fill)
    return out


def mixed_u64(n: int = 1_000_000_000, seed: int = 3) -> np.ndarray:
    """Equal thirds (the first takes the remainder) of three u64 families at
    uniformly random positions: the exact family counts of each CHUNK-sized
    piece are drawn hypergeometrically, then shuffled inside the piece, which
    places the thirds as a global shuffle would."""
    r = _rng(seed)
    left = np.array([n - 2 * (n // 3), n // 3, n // 3], dtype=np.int64)
    counts = []
    for lo in range(0, n, CHUNK):
        k = min(n, lo + CHUNK) - lo
        if k < left.sum():
            c0 = r.hypergeometric(left[0], left[1] + left[2], k) if left[0] else 0
            c1 = r.hypergeometric(left[1], left[2], k - c0) if left[1] and k > c0 else 0
            c = np.array([c0, c1, k - c0 - c1], dtype=np.int64)
        else:
            c = left.copy()
        left -= c
        counts.append(c)
    out = np.empty(n, dtype=np.uint64)

    def fill(c, lo, hi):
        g = _rng(seed, 1 + c)
        k0, k1, k2 = (int(v) for v in counts[c])
        v = np.empty(hi - lo, dtype=np.uint64)
        a = np.rint(g.normal(2.0 ** 40, 2.0 ** 36, size=k0))
        v[:k0] = np.clip(a, 0, 2.0 ** 63).astype(np.uint64)
        v[k0:k0 + k1] = np.rint(g.exponential(2.0 ** 30, size=k1)).astype(np.uint64)
        v[k0 + k1:] = g.integers(0, 2 ** 64, size=k2, dtype=np.uint64, endpoint=False) % np.uint64(10_000)
        g.shuffle(v)
        out[lo:hi] = v

    _chunked(n, fill)
    return out


def log_uniform_sizes(r: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    return np.floor(np.exp(r.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def zipf_dup(r: np.random.Generator, size: int, dup_ratio: float, s: float = 1.2,
             dtype=np.float64) -> np.ndarray:
    """`size` keys with an exact duplicate ratio: D = max(1, round((1-d)*size))
    distinct values, each placed once, the rest Zipf(s) over them, shuffled."""
    d = max(1, int(round((1.0 - dup_ratio) * size)))
    d = min(d, size)
    if dtype == np.float64:
        vals = r.lognormal(0.0, 1.0, size=d)
    else:
        vals = np.rint(r.exponential(2.0 ** 30, size=d)).astype(np.uint64)
    vals = np.unique(vals)                      # distinct by construction
    d = vals.size
    rest = size - d
    out = np.empty(size, dtype=vals.dtype)
    out[:d] = vals
    if rest:
        cdf = zipf_table(d, s)
        rank = np.minimum(np.searchsorted(cdf, r.random(rest), side="right"), d - 1)
        out[d:] = vals[rank]
    r.shuffle(out)
    return out


FAMILIES = ("uniform", "normal", "lognormal", "zipfdup")


@dataclass
class SegmentSpec:
    sizes: np.ndarray       # keys per segment
    family: np.ndarray      # index into FAMILIES
    dup_ratio: np.ndarray   # used by zipfdup
    seed: int

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.uint64)


def segment_spec(count: int = 10_000, seed: int = 4, lo: int = 1024, hi: int = 4_194_304) -> SegmentSpec:
    r = _rng(seed)
    sizes = log_uniform_sizes(r, count, lo, hi)
    fam = r.integers(0, len(FAMILIES), size=count)
    dup = r.uniform(0.0, 0.99, size=count)
    return SegmentSpec(sizes, fam, dup, seed)


def segment_keys(spec: SegmentSpec, i: int) -> np.ndarray:
    """Keys of segment i (f64), drawn from its own stream."""
    r = _rng(spec.seed, 1_000_000 + i)
    k = int(spec.sizes[i])
    fam = FAMILIES[int(spec.family[i])]
    if fam == "uniform":
        return r.random(k)
    if fam == "normal":
        return r.normal(0.0, 1.0, size=k)
    if fam == "lognormal":
        return r.lognormal(0.0, 1.0, size=k)
    return zipf_dup(r, k, float(spec.dup_ratio[i]))


def segments(spec: SegmentSpec, out: np.ndarray | None = None, workers: int | None = None) -> np.ndarray:
    """All segments back to back (each from its own stream, in threads)."""
    total = int(spec.sizes.sum())
    if out is None:
        out = np.empty(total, dtype=np.float64)
    off = spec.offsets

    def fill(i):
        out[int(off[i]):int(off[i + 1])] = segment_keys(spec, i)

    w = workers or _workers()
    if w == 1:
        for i in range(spec.sizes.size):
            fill(i)
    else:
        with ThreadPoolExecutor(w) as ex:
            list(ex.map(fill, range(spec.sizes.size)))
    return out


@dataclass
class RequestSpec:
    sizes: np.ndarray       # keys per request
    is_u64: np.ndarray      # bool: u64 (else f64)
    dup_ratio: np.ndarray
    arrival_s: np.ndarray   # Poisson arrival times (seconds from start)
    seed: int


def request_spec(count: int = 50_000, seed: int = 5, rate_per_s: float = 1000.0,
                 lo: int = 1024, hi: int = 67_108_864) -> RequestSpec:
    r = _rng(seed)
    sizes = log_uniform_sizes(r, count, lo, hi)
    is_u64 = r.random(count) < 0.5
    dup = r.uniform(0.0, 0.99, size=count)
    gaps = r.exponential(1.0 / rate_per_s, size=count)
    return RequestSpec(sizes, is_u64, dup, np.cumsum(gaps), seed)


def request_keys(spec: RequestSpec, i: int) -> np.ndarray:
    """Keys of request i: f64 lognormal(0,1) or u64 round(Exp(2^30)) values
    with the request's duplicate ratio."""
    r = _rng(spec.seed, 2_000_000 + i)
    dt = np.uint64 if spec.is_u64[i] else np.float64
    return zipf_dup(r, int(spec.sizes[i]), float(spec.dup_ratio[i]), dtype=dt)


# ------------------------------------------------- paper's synthetic families --

def root_dups(n: int) -> np.ndarray:
    """A[i] = i mod floor(sqrt(N))."""
    return (np.arange(n, dtype=np.uint64) % np.uint64(max(1, math.isqrt(n)))).astype(np.float64)


def two_dups(n: int) -> np.ndarray:
    """A[i] = (i^2 + N/2) mod N, in exact integer arithmetic."""
    i = np.arange(n, dtype=np.uint64)
    nn = np.uint64(n)
    sq = ((i % nn) * (i % nn)) % nn if n < (1 << 32) else np.array(
        [(int(x) * int(x)) % n for x in i], dtype=np.uint64)
    return ((sq + np.uint64(n // 2)) % nn).astype(np.float64)


def mix_gauss(n: int, seed: int = 6, k: int = 5) -> np.ndarray:
    """Mixture of k Gaussians with random means, deviations and weights."""
    r = _rng(seed)
    means = r.uniform(-100.0, 100.0, size=k)
    sds = r.uniform(0.5, 20.0, size=k)
    w = r.random(k)
    w /= w.sum()
    comp = r.choice(k, size=n, p=w)
    return r.normal(means[comp], sds[comp])


def paper_family(name: str, n: int, seed: int = 7) -> np.ndarray:
    r = _rng(seed)
    if name == "uniform":
        return r.uniform(0.0, float(n), size=n)
    if name == "normal":
        return r.normal(0.0, 1.0, size=n)
    if name == "lognormal":
        return r.lognormal(0.0, 0.5, size=n)
    if name == "chi_square":
        return r.chisquare(4.0, size=n)
    if name == "exponential":
        return r.exponential(1.0 / 2.0, size=n)
    if name == "root_dups":
        return root_dups(n)
    if name == "two_dups":
        return two_dups(n)
    if name == "mix_gauss":
        return mix_gauss(n, seed)
    if name.startswith("zipf"):
        # ranks 1..n: the universe is unstated; n ranks gives skew 0.9 the
        # paper's 72% duplicates (Sec. 3)
        skew = float(name[4:] or 0.9)
        ranks = np.searchsorted(zipf_table(n, skew), r.random(n), side="right")
        return ranks.astype(np.float64)
    raise KeyError(name)


def paper_family_large(name: str, n: int, seed: int = 7) -> np.ndarray:
    """paper_family for sizes up to 10^9, drawn CHUNK keys at a time in
    threads (each piece from its own stream, so the values do not depend on
    the thread count; they differ from paper_family's single stream)."""
    if n <= CHUNK:
        return paper_family(name, n, seed)
    out = np.empty(n, dtype=np.float64)
    if name in ("root_dups", "two_dups"):
        nn = np.uint64(n)
        root = np.uint64(max(1, math.isqrt(n)))

        def fill(c, lo, hi):
            i = np.arange(lo, hi, dtype=np.uint64)
            if name == "root_dups":
                out[lo:hi] = (i % root).astype(np.float64)
            else:       # n < 2^32 keeps i * i inside 64 bits
                out[lo:hi] = (((i * i) % nn + np.uint64(n // 2)) % nn).astype(np.float64)

        if name == "two_dups" and n >= (1 << 32):
            raise ValueError("two_dups needs n < 2^32")
        _chunked(n, fill)
        return out
    if name == "mix_gauss":
        r = _rng(seed)
        k = 5
        means = r.uniform(-100.0, 100.0, size=k)
        sds = r.uniform(0.5, 20.0, size=k)
        w = r.random(k)
        w /= w.sum()
    if name.startswith("zipf"):
        skew = float(name[4:] or 0.9)
        cdf = zipf_table(n, skew)

    def fill(c, lo, hi):
        g = _rng(seed, 1 + c)
        m = hi - lo
        if name == "uniform":
            out[lo:hi] = g.uniform(0.0, float(n), size=m)
        elif name == "normal":
            out[lo:hi] = g.normal(0.0, 1.0, size=m)
        elif name == "lognormal":
            out[lo:hi] = g.lognormal(0.0, 0.5, size=m)
        elif name == "chi_square":
            out[lo:hi] = g.chisquare(4.0, size=m)
        elif name == "exponential":
            out[lo:hi] = g.exponential(1.0 / 2.0, size=m)
        elif name == "mix_gauss":
            comp = g.choice(k, size=m, p=w)
            out[lo:hi] = g.normal(means[comp], sds[comp])
        elif name.startswith("zipf"):
            out[lo:hi] = np.searchsorted(cdf, g.random(m), side="right").astype(np.float64)
        else:
            raise KeyError(name)

    _chunked(n, fill)
    return out


def duplicate_ratio(a: np.ndarray) -> float:
    """Fraction of keys equal to an earlier key (1 - distinct / n)."""
    if a.size == 0:
        return 0.0
    return 1.0 - np.unique(a.view(np.uint64) if a.dtype == np.float64 else a).size / a.size
