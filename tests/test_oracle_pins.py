"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
examples of Alg. 1 / Alg. 2 (tests/golden), published generator outputs,
library sorting (numpy), brute force over tiny inputs, closed forms and
invariants the paper states.  No GPU needed.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import SPECIAL_F64, expected_sorted, ord_words, raw_words

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def q(expr: str) -> float:
    """Evaluate a hand-derived quotient from the golden file in IEEE double."""
    return float(eval(expr, {"__builtins__": {}}, {}))


# ----------------------------------------------------------------- sampling --

def test_splitmix64_published_outputs():
    g = GOLDEN["splitmix64"]
    L = oracle.lib()
    assert L.orc_splitmix64_at(0, 0) == int(g["seed0_first"], 16)
    assert [L.orc_splitmix64_at(1234567, t) for t in range(5)] == [int(v) for v in g["seed1234567_first5"]]


@pytest.mark.parametrize("n", [1, 7, 99, 100, 101, 12345, 1_000_000, 200_000_000, 10 ** 9, 2 ** 40 + 3])
def test_sample_size_is_ceil_one_percent(n):
    # Sec. 6.1: 1% sample; reading R16: m = max(1, ceil(n/100)).
    assert oracle.lib().orc_sample_size(n, 0.01, 0) == max(1, -(-n // 100))


def test_sample_size_cap():
    assert oracle.lib().orc_sample_size(10 ** 9, 0.01, 123) == 123


def test_sample_indices_in_range_and_uniform():
    n = 1000
    idx = np.array([oracle.lib().orc_sample_index(99, t, n) for t in range(20000)])
    assert idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx // 100, minlength=10)
    chi2 = ((counts - 2000.0) ** 2 / 2000.0).sum()
    assert chi2 < 40.0          # 9 dof; p < 1e-5 for a correct uniform sampler
    # index = floor(u * n / 2^64) for u the generator output (exact check on t = 0..9)
    for t in range(10):
        u = oracle.lib().orc_splitmix64_at(99, t)
        assert oracle.lib().orc_sample_index(99, t, n) == (u * n) >> 64


# -------------------------------------------------------------------- model --

def test_model_training_worked_example():
    g = GOLDEN["model_training"]
    m = oracle.train_sample(np.array(g["sample"]), g["leaves"])
    e = g["expected"]
    want = [q(e["xmin"]), q(e["xmax"]), q(e["rs"]), q(e["mfin"])]
    want += [q(v) for v in e["leaf0"]] + [q(v) for v in e["leaf1"]] + [q(v) for v in e["start"]]
    assert m.tolist() == want
    F = oracle.model_eval(m, g["leaves"], np.array(g["eval_x"]))
    assert F.tolist() == [q(v) for v in g["eval_F"]]


def _leaves(model):
    """X, y, ym, y1, ylo, yhi, s of the L leaf knots, then the start knot."""
    return tuple(model[4 + c::7] for c in range(7))


@pytest.mark.parametrize("family", ["uniform", "normal", "lognormal", "zipfdup", "u64mixed"])
def test_model_knots_are_exact_ecdf(family):
    # Sec. 2: the model returns the count of keys less than x, scaled; at a
    # knot X the sample counts below it and at it are known exactly:
    # y = #(< X)/m', ym = (#(< X) + #(<= X))/(2m'), y1 = #(<= X)/m', and the
    # segment above the knot starts from y1.
    r = np.random.default_rng(11)
    if family == "uniform":
        a = r.random(50_000)
    elif family == "normal":
        a = r.normal(size=50_000)
    elif family == "lognormal":
        a = r.lognormal(0, 2, size=50_000)
    elif family == "zipfdup":
        a = W.zipf_dup(r, 50_000, 0.9)
    else:
        a = W.mixed_u64(60_000, seed=5)
    L = 64
    model, idx = oracle.train(a, leaves=L)
    sample = a[idx.astype(np.int64)]
    sv = sample.astype(np.float64)
    m_fin = np.isfinite(sv).sum()
    assert model[3] == m_fin
    X, y, ym, y1, ylo, yhi, s = _leaves(model)
    assert X.size == L + 1
    assert X[L] == sv.min()                     # the start knot
    knots = np.flatnonzero(np.isfinite(X))
    assert knots.size >= 2
    assert np.all(np.diff(X[knots[:-1]]) > 0)   # leaf knots increase
    for k in knots:
        below = int((sv < X[k]).sum())
        upto = int((sv <= X[k]).sum())
        assert y[k] == below / m_fin
        assert y1[k] == upto / m_fin
        assert ym[k] == (below + upto) / (2 * m_fin)
        assert ylo[k] == (2 * upto - 1) / (2 * m_fin)       # mid-rank of the last copy
        assert X[k] in sv                       # knots are sample values
    if a.dtype == np.float64:
        Fk = oracle.model_eval(model, L, np.asarray(X[knots], dtype=np.float64))
        assert np.array_equal(Fk, ym[knots])
        # just above a knot (below the next one) F is at least the mid-rank
        # of the knot's last copy, just below it at most that of its first
        order = np.argsort(X[knots])
        kk = knots[order]
        lk = X[kk]
        above = np.nextafter(lk, np.inf)
        inside = above < np.append(lk[1:], np.inf)
        Fa = oracle.model_eval(model, L, above[inside])
        assert np.all(Fa >= ylo[kk][inside])
        below_k = np.nextafter(lk[1:], -np.inf)
        ok = below_k > lk[:-1]
        Fb = oracle.model_eval(model, L, below_k[ok])
        assert np.all(Fb <= ((2 * (y[kk[1:]] * m_fin) + 1) / (2 * m_fin))[ok])


def test_model_knot_is_the_most_repeated_value_nearby():
    # A leaf's knot is its most repeated sample value when that value holds
    # at least 1/L of the sample.  A leaf lies between the knots around it,
    # so no value that heavy sits strictly between two consecutive knots
    # unless one of them repeats at least as often; the most repeated value
    # of the whole sample is a knot.
    r = np.random.default_rng(14)
    a = W.zipf_dup(r, 60_000, 0.97)
    L = 48
    model, idx = oracle.train(a, leaves=L, sample_rate=0.2)
    sv = a[idx.astype(np.int64)]
    m = sv.size
    vals, mult = np.unique(sv, return_counts=True)
    X = _leaves(model)[0]
    knots = np.unique(X[np.isfinite(X)])
    km = {v: c for v, c in zip(vals, mult)}
    heavy = (mult >= 2) & (mult * L >= m)
    assert heavy.sum() >= 3
    for lo, hi in zip(knots[:-1], knots[1:]):
        inner = (vals > lo) & (vals < hi) & heavy
        if inner.any():
            assert mult[inner].max() <= max(km[lo], km[hi])
    assert vals[np.argmax(mult)] in knots
    # with no value that heavy every knot is its leaf's smallest value, so
    # no sample value lies strictly below the lowest leaf knot but above xmin
    u = np.random.default_rng(15).random(20_000)
    model, idx = oracle.train(u, leaves=L, sample_rate=0.2)
    su = u[idx.astype(np.int64)]
    Xu = _leaves(model)[0][:L]
    first_knot = Xu[np.isfinite(Xu)].min()
    assert first_knot == su.min()


def test_model_isolates_a_heavy_sample_value():
    # A value holding at least two buckets' worth of the sample falls strictly
    # between the keys below and above it: its level-0 bucket holds it alone.
    r = np.random.default_rng(13)
    f = 64
    heavy = 0.37
    a = np.concatenate([r.random(40_000), np.full(4_000, heavy)])
    r.shuffle(a)
    model, _ = oracle.train(a, leaves=32, sample_rate=0.05)
    b = oracle.bucket(model, 32, a, scale=f, offset=0, fanout=f)
    hb = b[a == heavy]
    assert np.all(hb == hb[0])
    assert not np.any((b == hb[0]) & (a != heavy))


@pytest.mark.parametrize("family", ["uniform", "lognormal", "zipfdup", "specials"])
def test_model_monotone_and_bounded(family):
    r = np.random.default_rng(12)
    if family == "uniform":
        a = r.random(20_000)
    elif family == "lognormal":
        a = r.lognormal(0, 2, size=20_000)
    elif family == "zipfdup":
        a = W.zipf_dup(r, 20_000, 0.95)
    else:
        a = np.concatenate([r.normal(size=5000) * 1e300, SPECIAL_F64, [np.nan, -np.nan, 1e-310]])
    for L in (1, 7, 100):
        model, _ = oracle.train(a, leaves=L, sample_rate=0.05)
        xs = np.sort(a[~np.isnan(a)])
        F = oracle.model_eval(model, L, xs)
        assert np.all(F >= 0.0) and np.all(F <= 1.0)
        assert np.all(np.diff(F) >= 0.0)


def test_model_close_to_cdf_on_uniform():
    # DKW: sup |ECDF - CDF| <= sqrt(ln(2/delta) / 2m) with prob 1 - delta.
    a = W.uniform_1e9grid(1_000_000, seed=1)
    model, idx = oracle.train(a)
    m = idx.size
    eps = math.sqrt(math.log(2 / 1e-6) / (2 * m))
    xs = np.linspace(0.0, 0.999, 2001)
    F = oracle.model_eval(model, 1000, xs)
    # interpolation between knots adds at most one leaf's share of the sample
    assert np.abs(F - xs).max() <= eps + 2.0 / 1000 + 1.0 / m


def test_model_nonfinite_routing():
    # Reading R20: negative non-finite keys predict 0, positive ones 1.
    a = np.array([1.0, 2.0, 3.0, 4.0])
    model = oracle.train_sample(a, 4)
    F = oracle.model_eval(model, 4, np.array([-np.inf, np.inf, np.nan, -np.nan]))
    assert F.tolist() == [0.0, 1.0, 1.0, 0.0]


def test_model_u64_rounds_to_nearest_even():
    # Reading R24: 2^53 and 2^53+1 are the same double, so the same prediction.
    s = np.array([0, 2 ** 52, 2 ** 53, 2 ** 60], dtype=np.uint64)
    model = oracle.train_sample(s, 4)
    F = oracle.model_eval(model, 4, np.array([2 ** 53, 2 ** 53 + 1], dtype=np.uint64))
    assert F[0] == F[1]


# ------------------------------------------------------- Alg. 1 / Defragment --

def test_partition_worked_example_level0():
    g = GOLDEN["partition_level0"]
    model = np.array(g["model"])
    out, sb, flog = oracle.partition(np.array(g["keys"]), model, g["leaves"], g["fanout"],
                                     g["frag_cap"], level=0)
    assert out.tolist() == g["after_partition"]
    assert sb.tolist() == g["S_B"]
    assert flog.tolist() == g["frag_log"]
    d = oracle.defragment(out, sb, g["fanout"], flog)
    assert d.tolist() == g["after_defragment"]


def test_partition_worked_example_level1():
    g0 = GOLDEN["partition_level0"]
    g = GOLDEN["partition_level1"]
    model = np.array(g0["model"])
    out, sb, flog = oracle.partition(np.array(g["keys"]), model, g0["leaves"], g0["fanout"],
                                     g0["frag_cap"], level=1, parent=g["parent"])
    assert out.tolist() == g["after_partition"]
    assert sb.tolist() == g["S_B"]
    assert flog.tolist() == g["frag_log"]
    assert oracle.defragment(out, sb, g0["fanout"], flog).tolist() == g["after_defragment"]


def test_counting_sort_worked_example():
    g0 = GOLDEN["partition_level0"]
    g = GOLDEN["counting_sort"]
    f = g0["fanout"]
    out = oracle.counting_sort(np.array(g["keys"]), np.array(g0["model"]), g0["leaves"],
                               float(f * f), float(g["parent"] * f + g["sub"]))
    assert out.tolist() == g["after_counting_sort"]
    fixed, moves = oracle.insertion_sort(out)
    assert fixed.tolist() == g["after_insertion_sort"]
    assert moves == g["insertion_moves"]


@pytest.mark.parametrize("f,c,n", [(4, 2, 37), (16, 5, 1000), (64, 100, 20_000), (1000, 100, 100_000)])
def test_partition_invariants(f, c, n):
    r = np.random.default_rng(f * 7 + c)
    a = np.concatenate([r.lognormal(0, 1, size=n - n // 4), np.full(n // 4, 0.75)])
    r.shuffle(a)
    model, _ = oracle.train(a, leaves=min(1000, f), sample_rate=0.05)
    L = min(1000, f)
    out, sb, flog = oracle.partition(a, model, L, f, c)
    # every key accounted for; copy-back is a permutation
    assert int(sb.sum()) == n
    assert np.array_equal(np.sort(raw_words(out)), np.sort(raw_words(a)))
    # full fragments hold exactly c keys; at most one partial fragment per bucket
    full = flog[flog[:, 1] == c]
    part = flog[flog[:, 1] < c]
    assert np.all(flog[:, 1] >= 1)
    assert len(np.unique(part[:, 0])) == len(part)
    assert len(flog) <= n // c + f
    # per-bucket fragment sizes add up to S_B
    per = np.bincount(flog[:, 0].astype(int), weights=flog[:, 1], minlength=f)
    assert np.array_equal(per.astype(np.uint64), sb)
    # defragmented buckets: each key predicts its bucket, buckets are ordered
    d = oracle.defragment(out, sb, f, flog)
    off = np.concatenate([[0], np.cumsum(sb)]).astype(int)
    b = oracle.bucket(model, L, d, float(f), 0, f)
    o = ord_words(d)
    prev_max = -1
    for i in range(f):
        seg = slice(off[i], off[i + 1])
        assert np.all(b[seg] == i)
        if off[i + 1] > off[i]:
            assert int(o[seg].min()) >= prev_max
            prev_max = int(o[seg].max())
    assert full.shape[0] >= 0


def test_write_head_never_passes_read_head_adversarial():
    # Sec. 4.2: overwritten slots were already scanned.  A run of keys that
    # fills one fragment after another is the tightest case.
    f, c = 8, 3
    a = np.repeat(np.linspace(0.0, 1.0, f, endpoint=False), 50)
    model = oracle.train_sample(np.linspace(0.0, 1.0, 64), 8)
    out, sb, flog = oracle.partition(a, model, 8, f, c)      # raises on a violation
    assert int(sb.sum()) == a.size


# ------------------------------------------------------------ Alg. 2 stages --

def test_stage_level0_invariants():
    a = W.zipf_lognormal(300_000, seed=9, distinct=300)
    f = 64
    st = oracle.stage_level0(a, fanout=f, leaves=64, frag_cap=10, with_sb1=True)
    sb = st["sb"]
    assert int(sb.sum()) == a.size
    keys = st["keys"]
    assert np.array_equal(np.sort(keys), np.sort(raw_words(a)))
    off = np.concatenate([[0], np.cumsum(sb)]).astype(int)
    o = ord_words(keys.view(np.float64))
    prev = -1
    for i in range(f):
        seg = o[off[i]:off[i + 1]]
        if seg.size:
            assert int(st["min"][i]) == int(seg.min())
            assert int(st["max"][i]) == int(seg.max())
            assert int(seg.min()) >= prev
            prev = int(seg.max())
        assert bool(st["homog"][i]) == (seg.size <= 1 or bool(np.all(seg == seg[0])))
        if not st["homog"][i]:
            assert int(st["sb1"][i].sum()) == seg.size
        else:
            assert int(st["sb1"][i].sum()) == 0
    assert st["homog"].sum() >= 1        # a Zipf input has all-equal buckets


# ------------------------------------------------------------- final result --

def _check(a, **kw):
    s, stt = oracle.sort(a, **kw)
    assert np.array_equal(raw_words(s), expected_sorted(a))
    return stt


CASES = {
    "uniform": lambda n, r: W.uniform_1e9grid(n, seed=int(r.integers(1 << 30))),
    "normal": lambda n, r: r.normal(size=n),
    "lognormal2": lambda n, r: r.lognormal(0, 2, size=n),
    "zipf": lambda n, r: W.zipf_lognormal(n, seed=int(r.integers(1 << 30)), distinct=max(2, n // 50)),
    "allequal": lambda n, r: np.full(n, 3.25),
    "twovalues": lambda n, r: r.choice([-0.0, 0.0], size=n),
    "specials": lambda n, r: r.choice(np.concatenate([SPECIAL_F64, [np.nan, -np.nan, 1.7976931348623157e308, -5e-324]]), size=n),
    "sorted": lambda n, r: np.arange(n, dtype=np.float64),
    "reverse": lambda n, r: np.arange(n, 0, -1, dtype=np.float64),
    "u64mixed": lambda n, r: W.mixed_u64(n, seed=int(r.integers(1 << 30))),
    "u64full": lambda n, r: r.integers(0, 2 ** 64, size=n, dtype=np.uint64, endpoint=False),
    "u64edges": lambda n, r: r.choice(np.array([0, 1, 2 ** 53 - 1, 2 ** 53, 2 ** 53 + 1, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64), size=n),
    "rootdups": lambda n, r: W.root_dups(n),
    "twodups": lambda n, r: W.two_dups(n),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 1000, 4097, 50_001])
def test_sort_equals_library_sort_paper_params(case, n):
    r = np.random.default_rng(n + 1)
    _check(CASES[case](n, r))


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("kw", [dict(fanout=4, frag_cap=2, leaves=4, small_n=1),
                                dict(fanout=16, frag_cap=3, leaves=8, small_n=1, s_max=20),
                                dict(fanout=256, frag_cap=16, leaves=256, s_max=2000)])
def test_sort_equals_library_sort_small_params(case, kw):
    r = np.random.default_rng(7)
    for n in (5, 97, 3000):
        _check(CASES[case](n, r), **kw)


def test_bruteforce_all_length6_sequences():
    # All 8^6 sequences over 8 special doubles, small parameters so that every
    # stage (fragments, level 1, counting sort, touch-up) runs.
    vals = SPECIAL_F64
    allseq = np.array(list(itertools.product(range(8), repeat=6)), dtype=np.int64)
    kw_lit = dict(fanout=4, frag_cap=2, leaves=4, small_n=1, sample_rate=0.5)
    kw_rec = dict(fanout=2, frag_cap=1, leaves=2, small_n=1, s_max=2, sample_rate=0.5, local_min_sample=2)
    L = oracle.lib()
    p_lit = oracle.params(oracle.F64, **kw_lit)
    p_rec = oracle.params(oracle.F64, **kw_rec)
    st = oracle.Stats()
    import ctypes
    buf = np.zeros(6, np.uint64)
    ptr = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    words = raw_words(vals)
    exp = expected_sorted(vals)
    rank = {int(w): i for i, w in enumerate(exp)}
    for p in (p_lit, p_rec):
        for row in allseq:
            buf[:] = words[row]
            assert L.orc_sort(ptr, 6, ctypes.byref(p), ctypes.byref(st)) == 0
            got = [rank[int(w)] for w in buf]
            assert got == sorted(row_rank for row_rank in (rank[int(w)] for w in words[row]))


def test_bruteforce_all_permutations_of_8():
    vals = np.array([-2.5, -1e-300, -0.0, 0.0, 1e-300, 1.0, 3.0, 1e300])
    exp = expected_sorted(vals)
    for kw in (dict(fanout=4, frag_cap=2, leaves=4, small_n=1, sample_rate=0.5),
               dict(fanout=2, frag_cap=1, leaves=2, small_n=1, s_max=2, sample_rate=0.5,
                    local_min_sample=2)):
        for perm in itertools.permutations(range(8)):
            s, _ = oracle.sort(vals[list(perm)], **kw)
            assert np.array_equal(raw_words(s), exp)


def test_nonfinite_total_order():
    a = np.array([np.nan, 1.0, -np.inf, -0.0, 0.0, np.inf, -np.nan, -1.0] * 40)
    s, _ = oracle.sort(a, fanout=8, frag_cap=2, leaves=4, small_n=1)
    o = ord_words(s)
    assert np.all(np.diff(o.astype(np.float64)) >= 0) or np.all(o[1:] >= o[:-1])
    assert np.array_equal(raw_words(s), expected_sorted(a))
    w = raw_words(s)
    assert np.isnan(s[0]) and (int(w[0]) >> 63) == 1          # -NaN first
    assert np.isnan(s[-1]) and (int(w[-1]) >> 63) == 0        # +NaN last


def test_no_progress_fallback_u64():
    # Reading R18: keys that round to one double cannot be separated by the
    # model; the highest-differing-bit split makes progress.  Its two children
    # (bit 0 = 0, then bit 0 = 1) are each all-equal, so the split alone puts
    # every key in place and the touch-up has nothing to move.
    a = np.array([2 ** 53, 2 ** 53 + 1] * 3000, dtype=np.uint64)
    np.random.default_rng(3).shuffle(a)
    st = _check(a, s_max=100, fanout=16, leaves=16)
    assert st.fallbacks >= 1
    assert st.touchup_moves == 0


def _split_spans(res: dict, keys: np.ndarray):
    """(min, max) order word of each non-empty child of a split, after
    checking that the split is a permutation with the stated sizes."""
    o = ord_words(res["keys"])
    assert np.array_equal(np.sort(o), np.sort(ord_words(keys)))
    sizes = res["sb"].astype(np.int64)
    assert int(sizes.sum()) == keys.size
    ends = np.cumsum(sizes)
    return [(int(o[e - z:e].min()), int(o[e - z:e].max())) for z, e in zip(sizes, ends) if z]


def _assert_ordered_and_separating(spans):
    # every key of a child is <= every key of the next non-empty child
    for (_, hi0), (lo1, _) in zip(spans, spans[1:]):
        assert hi0 <= lo1
    # progress: the range's minimum and maximum end in different children
    assert len(spans) >= 2


# 64 distinct u64 words within half an ulp of 2^62: they all round to the
# double 2^62, so no model separates them (reading R24).
NEAR_2_62 = np.uint64(2 ** 62) + np.arange(64, dtype=np.uint64)


def test_msd_split_digit_by_hand():
    # Reading R18 worked by hand: the words differ first at bit d = 5
    # (0 ^ 63 = 0b111111); with f = 16, b' = min(log2 16, d + 1) = 4 bits at
    # [2, 5], i.e. shift 2 and digit (w >> 2) & 15.  Value v goes to child
    # v // 4, so each child holds 4 values x 50 copies = 200 keys.
    a = np.repeat(NEAR_2_62, 50)
    np.random.default_rng(5).shuffle(a)
    res = oracle.split_stage(a, fanout=16, leaves=16)
    assert res["msd"] and res["shift"] == 2
    assert res["sb"].tolist() == [200] * 16
    _assert_ordered_and_separating(_split_spans(res, a))


def test_msd_split_on_sign_bit_by_hand():
    # f64 keys of both signs differ first at bit 63 of their order words;
    # b' = 4 at [60, 63]: the top nibbles of ord(-2.0) = 0x3FFF..., ord(-1.0)
    # = 0x400F..., ord(1.0) = 0xBFF0..., ord(2.0) = 0xC000... are 3, 4, 11, 12.
    a = np.repeat(np.array([2.0, -1.0, 1.0, -2.0]), [5, 7, 11, 13])
    np.random.default_rng(6).shuffle(a)
    res = oracle.split_stage(a, force_msd=True, fanout=16, leaves=16)
    assert res["msd"] and res["shift"] == 60
    expect = [0] * 16
    expect[3], expect[4], expect[11], expect[12] = 13, 7, 11, 5
    assert res["sb"].tolist() == expect
    _assert_ordered_and_separating(_split_spans(res, a))


@pytest.mark.parametrize("family", ["lognormal", "normal", "zipf"])
def test_local_split_children_ordered(family):
    # A local model split (reading R18) partitions by a monotone model: its
    # children are ordered, and a split that keeps its model makes progress
    # (no child holds more than 7/8 of the range).
    a = W.paper_family(family, 40_000, seed=17)
    res = oracle.split_stage(a, start=123, depth=3, fanout=64, leaves=64)
    assert not res["msd"]
    assert res["sb"].size == 64
    assert 8 * int(res["sb"].max()) <= 7 * a.size
    _assert_ordered_and_separating(_split_spans(res, a))


def test_msd_recursion_places_every_key_without_touchup():
    # Two levels of MSD splits (shift 2, then bits [0, 1]) leave every child
    # all-equal: the recursion alone sorts, so the touch-up moves nothing.
    a = np.repeat(NEAR_2_62, 200)
    np.random.default_rng(7).shuffle(a)
    st = _check(a, s_max=100, fanout=16, leaves=16)
    assert st.fallbacks >= 2
    assert st.touchup_moves == 0
    assert st.max_depth >= 3


def test_recursive_mode_bounds_touchup():
    # With recursion the touch-up has little left to do (P. 4.2: almost linear).
    a = W.zipf_lognormal(400_000, seed=21)
    lit = _check(a)
    rec = _check(a, s_max=4096)
    assert rec.touchup_moves <= lit.touchup_moves
    assert rec.touchup_moves < a.size


def test_touchup_moves_small_on_smooth_input():
    a = W.uniform_1e9grid(1_000_000, seed=1)
    st = _check(a)
    assert st.touchup_moves < 0.2 * a.size
    assert st.homogeneous >= 1 or st.counting_sorts >= 1


# --------------------------------------------------------------- generators --

def test_twodups_duplicate_ratio_near_paper():
    # Sec. 6.4 states 89% duplicates for TwoDups (N unstated).
    d = W.duplicate_ratio(W.two_dups(1_000_000))
    assert 0.80 <= d <= 0.96


def test_zipf_duplicate_ratio_near_paper():
    # Sec. 3: a Zipfian input of skew 0.9 holds 72% duplicates (universe
    # unstated; the generator draws ranks 1..n).
    d = W.duplicate_ratio(W.paper_family("zipf0.9", 1_000_000, seed=3))
    assert 0.62 <= d <= 0.80
    assert W.duplicate_ratio(W.paper_family("zipf0.5", 1_000_000, seed=3)) < d


def test_rootdups_duplicate_ratio_closed_form():
    n = 1_000_000
    assert W.duplicate_ratio(W.root_dups(n)) == 1.0 - math.isqrt(n) / n


def test_zipf_lognormal_shape():
    a = W.zipf_lognormal(2_000_000, seed=2)
    d = W.duplicate_ratio(a)
    assert d > 0.95
    _, counts = np.unique(a, return_counts=True)
    top = counts.max() / a.size
    # Zipf(1.2) over 1e5 ranks: rank 1 holds 1 / H(1e5, 1.2) of the mass
    h = float((np.arange(1, 100_001, dtype=np.float64) ** -1.2).sum())
    assert abs(top - 1.0 / h) < 0.01


def test_uniform_grid_duplicates_small():
    d = W.duplicate_ratio(W.uniform_1e9grid(1_000_000, seed=1))
    assert d < 0.002
