"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: bit-exact.  The sort result is unique (totalOrder / unsigned order), so
every output word must equal the oracle's; the stage hooks (model training,
one partition histogram) must match the oracle's stage data bit for bit too.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import SPECIAL_F64, expected_sorted, raw_words

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ls = pytest.importorskip("paper_2107_03290_amd")


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = ls.Sorter(0)
    yield s
    s.close()


def to_dev(a: np.ndarray):
    w = raw_words(a).view(np.int64).copy()
    t = torch.from_numpy(w).to("cuda:0")
    return t.view(torch.float64) if a.dtype == np.float64 else t


def words_of(t) -> np.ndarray:
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def gpu_sort(S, a, p=None):
    t = to_dev(a)
    S.sort_(t, p)
    torch.cuda.synchronize()
    return words_of(t)


def oracle_words(a, **kw):
    s, _ = oracle.sort(a, **kw)
    return raw_words(s)


def inputs(name, n, seed):
    r = np.random.default_rng(seed)
    if name == "uniform":
        return W.uniform_1e9grid(n, seed=seed)
    if name == "zipf":
        return W.zipf_lognormal(n, seed=seed, distinct=max(2, min(100_000, n // 20)))
    if name == "mixed_u64":
        return W.mixed_u64(n, seed=seed)
    if name == "normal":
        return r.normal(size=n)
    if name == "lognormal2":
        return r.lognormal(0, 2, size=n)
    if name == "allequal":
        return np.full(n, -7.25)
    if name == "twovalues":
        return r.choice([-0.0, 0.0], size=n)
    if name == "specials":
        return r.choice(np.concatenate([SPECIAL_F64, [np.nan, -np.nan, 1.7976931348623157e308]]), size=n)
    if name == "u64full":
        return r.integers(0, 2 ** 64, size=n, dtype=np.uint64, endpoint=False)
    if name == "u64edges":
        return r.choice(np.array([0, 1, 2 ** 53 - 1, 2 ** 53, 2 ** 53 + 1, 2 ** 63, 2 ** 64 - 1],
                                 dtype=np.uint64), size=n)
    if name == "sorted":
        return np.arange(n, dtype=np.float64)
    if name == "reverse":
        return np.arange(n, 0, -1, dtype=np.float64)
    if name == "twodups":
        return W.two_dups(n)
    if name == "rootdups":
        return W.root_dups(n)
    raise KeyError(name)


NAMES = ["uniform", "zipf", "mixed_u64", "normal", "lognormal2", "allequal", "twovalues", "specials",
         "u64full", "u64edges", "sorted", "reverse", "twodups", "rootdups"]


# --------------------------------------------------------------- stage hooks --

@pytest.mark.parametrize("name,n", [("uniform", 1_000_000), ("zipf", 400_000), ("mixed_u64", 300_000),
                                    ("specials", 50_000), ("lognormal2", 100_000), ("allequal", 20_000)])
@pytest.mark.parametrize("leaves", [1000, 1024, 7])
def test_model_training_bit_exact(S, name, n, leaves):
    a = inputs(name, n, 3)
    p = ls.params(leaves=leaves)
    g = S.model_train(to_dev(a), p)
    o, _ = oracle.train(a, leaves=leaves, seed=p.seed)
    assert np.array_equal(g.view(np.uint64), o.view(np.uint64))


@pytest.mark.parametrize("name,n", [("uniform", 1_000_000), ("zipf", 500_000), ("mixed_u64", 300_000),
                                    ("specials", 30_000)])
@pytest.mark.parametrize("fanout", [1000, 1024, 16])
def test_level0_histogram_bit_exact(S, name, n, fanout):
    a = inputs(name, n, 4)
    model, _ = oracle.train(a, leaves=1000)
    st = oracle.stage_level0(a, model=model, fanout=fanout, leaves=1000)
    c, lo, hi = S.stage_hist(to_dev(a), model, 1000, float(fanout), 0, fanout)
    assert np.array_equal(c, st["sb"])
    nz = c > 0
    assert np.array_equal(lo[nz], st["min"][nz]) and np.array_equal(hi[nz], st["max"][nz])


def test_level1_histograms_bit_exact(S):
    a = inputs("zipf", 300_000, 5)
    f = 64
    model, _ = oracle.train(a, leaves=64)
    st = oracle.stage_level0(a, model=model, fanout=f, leaves=64, with_sb1=True)
    off = np.concatenate([[0], np.cumsum(st["sb"])]).astype(np.int64)
    keys = st["keys"].view(np.float64)
    checked = 0
    for i in range(f):
        if st["homog"][i] or off[i + 1] - off[i] < 2:
            continue
        c, _, _ = S.stage_hist(to_dev(keys[off[i]:off[i + 1]]), model, 64, float(f * f), i * f, f)
        assert np.array_equal(c, st["sb1"][i]), i
        checked += 1
    assert checked >= 5


# ---------------------------------------------------------------- end to end --

@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4095, 4096, 4097, 100_003, 1_000_000])
def test_sort_matches_oracle(S, name, n):
    a = inputs(name, n, n + 17)
    got = gpu_sort(S, a)
    assert np.array_equal(got, expected_sorted(a))
    if 0 < n <= 200_000:
        assert np.array_equal(got, oracle_words(a, s_max=4096))


@pytest.mark.parametrize("kw", [dict(fanout=2), dict(fanout=16, leaves=8), dict(fanout=1000, leaves=1000),
                                dict(fanout=4096, leaves=256, tile=4096), dict(tile=1024), dict(tile=8192),
                                dict(tile=8192, fanout=2048, leaves=256), dict(tile=4096),
                                dict(base_threshold=2), dict(base_threshold=64, fanout=8),
                                dict(base_threshold=4096, fanout=64), dict(sample_rate=0.5),
                                dict(sample_cap=100), dict(leaves=1)])
@pytest.mark.parametrize("name", ["uniform", "zipf", "mixed_u64", "specials", "twovalues"])
def test_parameters_never_change_the_result(S, kw, name):
    a = inputs(name, 150_000, 23)
    got = gpu_sort(S, a, ls.params(**kw))
    assert np.array_equal(got, expected_sorted(a))


def test_wide_tile_rounds_match_the_definition(S):
    # the automatic tile scatters rounds of at least 2^25 keys in 8192-key
    # tiles (the round-0 task here, and the over-full buckets after it);
    # a fixed 4096-key tile must give the same words
    # with the model (1024 leaves) in LDS beside it, fanout 1600 still leaves
    # room for the wide tile (8192 * 10 + 1600 * 24 + 43080 bytes, the most a
    # wide tile may take), fanouts 2048 and 4096 do not (those rounds keep
    # smaller tiles)
    a = W.zipf_lognormal((1 << 25) + 12_345, seed=14, distinct=400_000)
    want = expected_sorted(a)
    for kw in (dict(), dict(tile=4096), dict(fanout=1600), dict(fanout=2048), dict(fanout=4096, leaves=512)):
        print("wide tile n=%d params=%s" % (a.size, kw), flush=True)
        got = gpu_sort(S, a, ls.params(**kw))
        assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["zipf_f64", "mixed_u64"])
def test_12288_key_tile_matches_the_definition(S, name):
    # with at most 512 leaves the automatic tile of rounds of at least 2^25
    # keys is 12,288 keys (32-bit cursors) up to fanout 1202, the most its LDS
    # holds beside a 512-leaf model (12288 * 10 + 1202 * 16 + 21576 bytes);
    # fanout 1300 keeps the smaller tiles
    n = (1 << 25) + 54_321
    a = (W.zipf_lognormal(n, seed=15, distinct=400_000) if name == "zipf_f64"
         else W.mixed_u64(n, seed=16))
    want = expected_sorted(a)
    for kw in (dict(leaves=512), dict(leaves=512, fanout=1202), dict(leaves=256, fanout=1000),
               dict(leaves=512, fanout=1300)):
        print("12288-key tile %s n=%d params=%s" % (name, n, kw), flush=True)
        got = gpu_sort(S, a, ls.params(**kw))
        assert np.array_equal(got, want)


def test_tile_that_does_not_fit_shrinks(S):
    # 8192- and 4096-key tiles with 4096 buckets and the 1024-leaf model need
    # more LDS than one workgroup has: the tile is halved until it fits
    a = inputs("zipf", 3_000_000, 12)
    for kw in (dict(tile=8192, fanout=4096), dict(tile=4096, fanout=4096, base_threshold=4096)):
        assert np.array_equal(gpu_sort(S, a, ls.params(**kw)), expected_sorted(a))
    t = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ls.LsortError):
        S.sort_(t, ls.params(tile=3000))


def test_device_bytes_and_trim(S):
    # the context keeps its work buffers (a key-sized scratch among them)
    # between sorts; trim frees them and the next sort allocates them again
    a = inputs("uniform", 1_000_000, 13)
    assert np.array_equal(gpu_sort(S, a), expected_sorted(a))
    assert S.device_bytes() >= a.size * 8
    S.trim()
    assert S.device_bytes() == 0
    assert np.array_equal(gpu_sort(S, a), expected_sorted(a))
    assert S.device_bytes() >= a.size * 8


def test_profile_all_classes_and_one_class(S):
    # every class timed, then the scatter alone; neither changes the result
    a = inputs("zipf", 2_000_000, 31)
    want = expected_sorted(a)
    S.profile_reset()
    assert np.array_equal(gpu_sort(S, a, ls.params(flags=ls.FLAG_PROFILE)), want)
    full = S.profile()
    for k in ("train", "hist", "scan", "classify", "scatter", "base", "touchup"):
        assert full[k][0] > 0 and full[k][1] > 0, k
    rounds = S.last_stats()["rounds"]
    assert full["scatter"][1] == rounds and full["hist"][1] == rounds
    assert full["scatter"][2] > 0
    S.profile_reset()
    only = ls.FLAG_PROFILE | ls.FLAG_PROFILE_ONLY(ls.KERNEL_CLASSES.index("scatter"))
    assert np.array_equal(gpu_sort(S, a, ls.params(flags=only)), want)
    one = S.profile()
    # (local models sample by position, so the round count may differ between two sorts)
    assert one["scatter"][1] == S.last_stats()["rounds"] and one["scatter"][2] > 0
    assert all(one[k][1] == 0 for k in ls.KERNEL_CLASSES if k != "scatter")
    # each class alone: its own launches only, and the same words
    for k, name in enumerate(ls.KERNEL_CLASSES):
        S.profile_reset()
        got = gpu_sort(S, a, ls.params(flags=ls.FLAG_PROFILE | ls.FLAG_PROFILE_ONLY(k)))
        assert np.array_equal(got, want), name
        prof = S.profile()
        assert prof[name][1] > 0 or full[name][1] == 0, name
        assert all(prof[c][1] == 0 for c in ls.KERNEL_CLASSES if c != name), name
    t = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ls.LsortError):
        S.sort_(t, ls.params(flags=ls.FLAG_PROFILE | (9 << 8)))


def test_debug_touchup_full_check(S):
    a = inputs("zipf", 300_000, 8)
    got = gpu_sort(S, a, ls.params(flags=ls.FLAG_DEBUG_TOUCHUP))
    assert np.array_equal(got, expected_sorted(a))
    assert S.last_stats()["seams_repaired"] == 0


def test_touchup_repairs_non_monotone_predictions(S):
    # Test hook: predictions are perturbed so buckets overlap; the touch-up
    # must detect the out-of-order seams and repair the result.
    a = inputs("uniform", 200_000, 9)
    got = gpu_sort(S, a, ls.params(flags=ls.FLAG_NONMONOTONE))
    assert np.array_equal(got, expected_sorted(a))
    assert S.last_stats()["seams_repaired"] > 0
    assert S.sync() & ls.DEV_SEAM_REPAIRED


def test_no_progress_fallback(S):
    a = np.array([2 ** 53, 2 ** 53 + 1, 2 ** 53 + 2] * 40_000, dtype=np.uint64)
    np.random.default_rng(1).shuffle(a)
    got = gpu_sort(S, a, ls.params(fanout=64))
    assert np.array_equal(got, expected_sorted(a))


def test_repeat_is_identical(S):
    a = inputs("zipf", 500_000, 10)
    g1 = gpu_sort(S, a)
    g2 = gpu_sort(S, a)
    assert np.array_equal(g1, g2)


# ----------------------------------------------------------------- segmented --

def test_segments_equal_single_sorts(S):
    spec = W.segment_spec(60, seed=31, lo=1, hi=200_000)
    keys = W.segments(spec)
    off = spec.offsets
    t = to_dev(keys)
    S.sort_segments_(t, off)
    torch.cuda.synchronize()
    got = words_of(t)
    for i in range(off.size - 1):
        seg = keys[int(off[i]):int(off[i + 1])]
        assert np.array_equal(got[int(off[i]):int(off[i + 1])], expected_sorted(seg)), i


def test_segments_mixed_dtypes_and_empty(S):
    r = np.random.default_rng(5)
    parts = [r.normal(size=10_000), np.array([], dtype=np.float64), r.lognormal(size=7),
             r.normal(size=300_000), np.array([1.5]), W.zipf_dup(r, 50_000, 0.9)]
    u = [W.mixed_u64(40_000, seed=2), r.integers(0, 2 ** 64, size=9_000, dtype=np.uint64, endpoint=False)]
    words = [raw_words(p) for p in parts] + [raw_words(x) for x in u]
    dts = [ls.F64] * len(parts) + [ls.U64] * len(u)
    allw = np.concatenate(words)
    off = np.concatenate([[0], np.cumsum([w.size for w in words])])
    t = torch.from_numpy(allw.view(np.int64).copy()).to("cuda:0")
    S.sort_segments_(t, off, dts)
    torch.cuda.synchronize()
    got = words_of(t)
    for i, p in enumerate(parts + u):
        assert np.array_equal(got[off[i]:off[i + 1]], expected_sorted(p)), i


def test_sort_arrays_separate_buffers(S):
    r = np.random.default_rng(6)
    arrs = [r.normal(size=int(s)) for s in (5, 5000, 70_000, 1)] + [W.mixed_u64(30_000, seed=3)]
    ts = [to_dev(a) for a in arrs]
    S.sort_arrays_(ts)
    torch.cuda.synchronize()
    for a, t in zip(arrs, ts):
        assert np.array_equal(words_of(t), expected_sorted(a))


# --------------------------------------------------------------- error paths --

def test_invalid_arguments_rejected(S):
    lib = ls.lib()
    assert lib.ls_sort_f64(S._ctx, None, 5, None, None) == 1
    bad = ls.params()
    bad.fanout = 1
    t = to_dev(np.zeros(10))
    assert lib.ls_sort_f64(S._ctx, t.data_ptr(), 10, None, bad) == 1
    bad = ls.params()
    bad.struct_size = 7
    assert lib.ls_sort_f64(S._ctx, t.data_ptr(), 10, None, bad) == 1
    import ctypes
    off = (ctypes.c_uint64 * 3)(0, 6, 4)
    assert lib.ls_sort_segments(S._ctx, 1, t.data_ptr(), off, 2, None, None, None) == 1
    assert lib.ls_sort_f64(S._ctx, t.data_ptr() + 4, 2, None, None) == 1     # misaligned
