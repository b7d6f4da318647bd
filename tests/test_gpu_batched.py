"""Batched segments and the autotuner, through the C ABI.

Each segment of a batch must come out exactly as its plain-definition sort
(a library sort of the order words), whatever the batch around it and
whatever parameters the autotuner picks.
"""
from concurrent.futures import ThreadPoolExecutor

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


def upload(a: np.ndarray):
    w = raw_words(a).view(np.int64)
    t = torch.empty(a.size, dtype=torch.int64, device="cuda:0")
    step = 1 << 26
    for lo in range(0, a.size, step):
        t[lo:lo + step].copy_(torch.from_numpy(w[lo:lo + step]))
    return t.view(torch.float64) if a.dtype == np.float64 else t


def download(t) -> np.ndarray:
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def check_segments(keys: np.ndarray, got: np.ndarray, off: np.ndarray, workers: int = 16):
    def one(i):
        lo, hi = int(off[i]), int(off[i + 1])
        return np.array_equal(got[lo:hi], expected_sorted(keys[lo:hi]))

    with ThreadPoolExecutor(workers) as ex:
        ok = list(ex.map(one, range(off.size - 1)))
    bad = [i for i, v in enumerate(ok) if not v]
    assert not bad, "segments differ: %s" % bad[:10]


def small_spec(count, seed, hi=300_000):
    return W.segment_spec(count=count, seed=seed, lo=1, hi=hi)


def test_autotune_keeps_input_and_picks_a_candidate(S):
    spec = small_spec(60, seed=21)
    keys = W.segments(spec)
    off = spec.offsets
    t = upload(keys)
    before = download(t)
    best, results = S.autotune([t], offsets=off, reps=1)
    torch.cuda.synchronize()
    assert np.array_equal(download(t), before)          # tuning works on a copy
    assert len(results) == 24
    assert {r["tile"] for r in results} == {2048, 0}         # 0: the automatic tile
    run = [r for r in results if r["ms"] >= 0]
    assert run, results
    fastest = min(run, key=lambda r: r["ms"])
    assert (best.fanout, best.tile, best.base_threshold) == \
        (fastest["fanout"], fastest["tile"], fastest["base_threshold"])
    S.sort_segments_(t, off, p=best)
    torch.cuda.synchronize()
    check_segments(keys, download(t), off)


def test_autotune_single_array_and_cache(S, tmp_path):
    a = W.zipf_lognormal(2_000_000, seed=5, distinct=5000)
    t = upload(a)
    cache = ls.TuneCache(str(tmp_path / "tune.json"))
    p1 = cache.tuned(S, [t], reps=1)
    again = ls.TuneCache(str(tmp_path / "tune.json"))          # read back from the file
    p2 = again.tuned(S, [t], reps=1)
    assert (p1.fanout, p1.tile, p1.base_threshold) == (p2.fanout, p2.tile, p2.base_threshold)
    S.sort_(t, p1)
    torch.cuda.synchronize()
    assert np.array_equal(download(t), expected_sorted(a))


@pytest.mark.parametrize("fanout,tile,base", [(512, 2048, 1024), (4096, 4096, 4096), (1024, 2048, 2048)])
def test_every_candidate_gives_the_same_batch(S, fanout, tile, base):
    spec = small_spec(200, seed=22, hi=2_000_000)
    keys = W.segments(spec)
    off = spec.offsets
    t = upload(keys)
    S.sort_segments_(t, off, p=ls.params(fanout=fanout, tile=tile, base_threshold=base))
    torch.cuda.synchronize()
    check_segments(keys, download(t), off)


def test_batched_equals_plain_per_segment(S):
    spec = small_spec(300, seed=23, hi=1_000_000)
    keys = W.segments(spec)
    off = spec.offsets
    tb = upload(keys)
    tp = tb.clone()
    S.sort_segments_(tb, off)
    for i in range(off.size - 1):
        S.sort_(tp[int(off[i]):int(off[i + 1])])
    torch.cuda.synchronize()
    assert torch.equal(tb.view(torch.int64), tp.view(torch.int64))
    check_segments(keys, download(tb), off)


@pytest.mark.slow
def test_ten_thousand_segments_full_size(S):
    """The full batch: 10,000 segments, about 5.1e9 keys (41 GB), every
    segment checked against the plain definition."""
    spec = W.segment_spec()
    keys = W.segments(spec)
    off = spec.offsets
    t = upload(keys)
    S.sort_segments_(t, off)
    torch.cuda.synchronize()
    got = download(t)
    del t
    torch.cuda.empty_cache()
    check_segments(keys, got, off)
