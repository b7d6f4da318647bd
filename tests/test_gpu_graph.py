"""Graph mode (LS_FLAG_GRAPH), through the C ABI.

A batch that runs as a replay of a captured HIP graph must come out exactly
as the plain-definition sort of each segment (a library sort of the order
words), and exactly as the host-driven pipeline sorts it.  (The round
statistics may differ between two runs of either path: the order of equal
bucket keys after a scatter is not fixed, and local models sample by
position.)  The graph of a size class is captured once and replayed with new
inputs, so every case runs several replays with host-driven sorts (and their
reallocations and task-list swaps) in between, and checks each replay.
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import expected_sorted, raw_words

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


def upload(words: np.ndarray):
    return torch.from_numpy(words.view(np.int64).copy()).to("cuda:0")


def download(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def batch(count, seed, lo=1, hi=200_000):
    spec = W.segment_spec(count=count, seed=seed, lo=lo, hi=hi)
    keys = W.segments(spec, workers=8)
    return keys, spec.offsets


def sort_batch(S, keys, off, p, dtypes=None):
    """Sort the segments of one batch; returns the words and the stats."""
    t = upload(raw_words(keys))
    S.sort_segments_(t.view(torch.float64), off, dtypes=dtypes, p=p)
    torch.cuda.synchronize()
    return download(t), S.last_stats()


def check(keys, got, off, dtypes=None):
    for i in range(off.size - 1):
        lo, hi = int(off[i]), int(off[i + 1])
        seg = keys[lo:hi]
        if dtypes is not None and dtypes[i] == ls.U64:
            seg = seg.view(np.uint64)
        want = raw_words(expected_sorted(seg))
        assert np.array_equal(got[lo:hi], want), "segment %d (%d keys) differs" % (i, hi - lo)


GRAPH = dict(flags=0x10)


def test_graph_flag_value():
    assert ls.FLAG_GRAPH == GRAPH["flags"]


@pytest.mark.parametrize("seed", [11, 12])
def test_graph_replays_match_definition_and_eager(S, seed):
    # four batches of the same size class, each checked; a host-driven sort
    # of a larger array between replays reallocates buffers (recapture)
    for rep in range(4):
        keys, off = batch(40, seed * 100 + rep)
        print("graph replay seed=%d rep=%d keys=%d segments=%d" % (seed, rep, keys.size, off.size - 1), flush=True)
        got, _ = sort_batch(S, keys, off, ls.params(**GRAPH))
        check(keys, got, off)
        ref, _ = sort_batch(S, keys, off, ls.params())
        assert np.array_equal(got, ref)
        if rep == 1:
            big = W.zipf_lognormal(6_000_000 + seed, seed=seed, distinct=50_000)
            t = upload(raw_words(big))
            S.sort_(t.view(torch.float64))
            torch.cuda.synchronize()
            assert np.array_equal(download(t), raw_words(expected_sorted(big)))


def test_graph_single_arrays_and_duplicates(S):
    p = ls.params(**GRAPH)
    cases = [W.zipf_lognormal(3_000_000, seed=3, distinct=20_000), W.root_dups(1 << 20), W.two_dups(1 << 20),
             np.full(1 << 18, 2.5), W.paper_family("mix_gauss", 1 << 21)]
    for rep in range(2):
        for a in cases:
            print("graph single n=%d rep=%d" % (a.size, rep), flush=True)
            off = np.array([0, a.size], dtype=np.uint64)
            got, _ = sort_batch(S, a, off, p)
            check(a, got, off)


def test_graph_small_and_empty_arrays_and_mixed_dtypes(S):
    # only base-case groups (no partition task), empty segments, u64 words
    r = np.random.default_rng(5)
    sizes = r.integers(0, 8000, size=300)
    sizes[::17] = 0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = r.normal(size=int(off[-1]))
    dts = [ls.U64 if i % 3 == 0 else ls.F64 for i in range(sizes.size)]
    p = ls.params(**GRAPH)
    for rep in range(3):
        print("graph small arrays rep=%d" % rep, flush=True)
        got, _ = sort_batch(S, keys, off, p, dtypes=dts)
        check(keys, got, off, dtypes=dts)
        keys = r.normal(size=int(off[-1]))


def test_graph_two_classes_alternate(S):
    p = ls.params(**GRAPH)
    small = batch(12, 31, hi=40_000)
    large = batch(30, 32, hi=300_000)
    for rep in range(3):
        for keys, off in (small, large):
            print("graph class keys=%d rep=%d" % (keys.size, rep), flush=True)
            got, _ = sort_batch(S, keys, off, p)
            check(keys, got, off)


def test_graph_deep_batch_continues_on_the_host(S):
    # fanout 4 and base threshold 64 need more rounds than one replay holds
    a = W.paper_family("uniform", 1 << 17, seed=9)
    off = np.array([0, a.size], dtype=np.uint64)
    p = ls.params(fanout=4, base_threshold=64, **GRAPH)
    for rep in range(2):
        print("graph deep rep=%d" % rep, flush=True)
        got, st = sort_batch(S, a, off, p)
        check(a, got, off)
        assert st["rounds"] > 4
        ref, _ = sort_batch(S, a, off, ls.params(fanout=4, base_threshold=64))
        assert np.array_equal(got, ref)


def test_graph_replay_after_task_list_swaps(S):
    # Host-driven rounds swap the context's two task lists.  With fanout 4
    # and base threshold 128 a 2^17-key sort takes five rounds: a replay
    # continues on the host for one round (one swap) and a host-driven sort
    # swaps five times, so every replay below starts with the lists traded
    # since the capture or since the last replay, and must still continue
    # from the list it wrote.
    p = ls.params(fanout=4, base_threshold=128, **GRAPH)
    e = ls.params(fanout=4, base_threshold=128)
    for rep in range(3):
        a = W.paper_family("uniform", 1 << 17, seed=20 + rep)
        off = np.array([0, a.size], dtype=np.uint64)
        print("graph after swaps rep=%d" % rep, flush=True)
        got, st = sort_batch(S, a, off, p)
        check(a, got, off)
        assert st["rounds"] > 4
        b = W.paper_family("normal", 1 << 17, seed=40 + rep)
        got_b, _ = sort_batch(S, b, off, e)
        check(b, got_b, off)


def test_graph_touchup_repair(S):
    # the test hook puts buckets out of order; the replay's touch-up must
    # find the seams and the host-driven repair pass fix them
    a = W.zipf_lognormal(2_000_000, seed=4, distinct=30_000)
    off = np.array([0, a.size], dtype=np.uint64)
    p = ls.params(flags=0x10 | ls.FLAG_NONMONOTONE)
    got, st = sort_batch(S, a, off, p)
    check(a, got, off)
    assert st["seams_repaired"] > 0
    assert S.sync() & ls.DEV_SEAM_REPAIRED


def test_graph_flag_combinations_and_classes(S):
    # profiling and the full touch-up check run host-driven; a batch above
    # 2^22 keys runs host-driven; 100 arrays use the 128-array class
    keys, off = batch(40, 77)
    for flags in (0x10 | ls.FLAG_PROFILE, 0x10 | ls.FLAG_DEBUG_TOUCHUP):
        print("graph flags=%#x" % flags, flush=True)
        S.profile_reset()
        got, st = sort_batch(S, keys, off, ls.params(flags=flags))
        check(keys, got, off)
        assert st["seams_repaired"] == 0
        if flags & ls.FLAG_PROFILE:
            assert S.profile()["scatter"][1] > 0
    big, off_big = batch(30, 78, lo=100_000, hi=400_000)
    assert int(off_big[-1]) > (1 << 22)
    print("graph large batch keys=%d" % big.size, flush=True)
    got, _ = sort_batch(S, big, off_big, ls.params(**GRAPH))
    check(big, got, off_big)
    many, off_many = batch(100, 79, hi=60_000)
    for rep in range(2):
        print("graph 100 arrays rep=%d" % rep, flush=True)
        got, _ = sort_batch(S, many, off_many, ls.params(**GRAPH))
        check(many, got, off_many)
