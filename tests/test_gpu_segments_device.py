"""ls_sort_segments_device: a batch described by device offsets and dtypes,
round 0 prepared on the device.  Bar: bit-exact against the definition and
word for word equal to the host-described ls_sort_segments of the same
batch, with the same rounds, tasks and all-equal buckets."""
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


def words_of(t) -> np.ndarray:
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def dev(a: np.ndarray, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).to("cuda:0")


def same_pipeline(a, b):
    # (the number of base-case groups may differ from run to run: groups are
    # formed by concurrent workgroups)
    return all(a[k] == b[k] for k in ("rounds", "tasks", "fill_buckets", "fill_keys", "max_level"))


def run_both(S, allw, off, dts=None, p=None, f64=False):
    host = torch.from_numpy(allw.view(np.int64).copy()).to("cuda:0")
    if f64:
        host = host.view(torch.float64)
    devt = host.clone()
    S.sort_segments_(host, off, dts, p)
    torch.cuda.synchronize()
    st_host = S.last_stats()
    d_off = dev(np.asarray(off, dtype=np.int64), np.int64)
    d_dt = dev(np.asarray(dts, dtype=np.uint8), np.uint8) if dts is not None else None
    S.sort_segments_device_(devt, d_off, d_dt, p)
    torch.cuda.synchronize()
    st_dev = S.last_stats()
    return words_of(host), words_of(devt), st_host, st_dev


def test_device_offsets_small_first(S):
    spec = W.segment_spec(20, seed=61, lo=1, hi=100_000)
    keys = W.segments(spec)
    print("device offsets: %d segments, %d keys" % (spec.offsets.size - 1, keys.size), flush=True)
    assert keys.dtype == np.float64
    h, d, sh, sd = run_both(S, raw_words(keys), spec.offsets, f64=True)
    assert np.array_equal(h, d) and same_pipeline(sh, sd)
    for i in range(spec.offsets.size - 1):
        lo, hi = int(spec.offsets[i]), int(spec.offsets[i + 1])
        assert np.array_equal(d[lo:hi], expected_sorted(keys[lo:hi])), i


@pytest.mark.parametrize("count,hi", [(1, 10), (7, 3_000), (300, 200_000), (2500, 20_000), (40, 4_000_000)])
def test_device_offsets_equal_host_offsets(S, count, hi):
    spec = W.segment_spec(count, seed=62 + count, lo=1, hi=hi)
    keys = W.segments(spec)
    h, d, sh, sd = run_both(S, raw_words(keys), spec.offsets, f64=keys.dtype == np.float64)
    assert np.array_equal(h, d)
    assert same_pipeline(sh, sd)
    for i in (0, count // 2, count - 1):
        lo, hi2 = int(spec.offsets[i]), int(spec.offsets[i + 1])
        assert np.array_equal(d[lo:hi2], expected_sorted(keys[lo:hi2])), i


def test_device_offsets_mixed_dtypes_empty_and_params(S):
    r = np.random.default_rng(7)
    parts = [r.normal(size=10_000), np.array([], dtype=np.float64), r.lognormal(size=7),
             r.normal(size=300_000), np.array([1.5]), W.zipf_dup(r, 50_000, 0.9)]
    u = [W.mixed_u64(40_000, seed=2), r.integers(0, 2 ** 64, size=9_000, dtype=np.uint64, endpoint=False)]
    words = [raw_words(p) for p in parts] + [raw_words(x) for x in u]
    dts = [ls.F64] * len(parts) + [ls.U64] * len(u)
    allw = np.concatenate(words)
    off = np.concatenate([[0], np.cumsum([w.size for w in words])])
    for p in (None, ls.params(fanout=64, base_threshold=512), ls.params(flags=ls.FLAG_INPLACE)):
        h, d, sh, sd = run_both(S, allw, off, dts, p)
        assert np.array_equal(h, d) and same_pipeline(sh, sd)
        for i, x in enumerate(parts + u):
            assert np.array_equal(d[off[i]:off[i + 1]], expected_sorted(x)), i


def test_device_offsets_empty_batch_and_invalid(S):
    t = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    S.sort_segments_device_(t, dev(np.array([0], dtype=np.int64), np.int64))
    S.sort_segments_device_(t, dev(np.array([0, 0, 16], dtype=np.int64), np.int64))
    torch.cuda.synchronize()
    with pytest.raises(ls.LsortError) as e:        # decreasing offsets, found on the device
        S.sort_segments_device_(t, dev(np.array([0, 9, 4, 16], dtype=np.int64), np.int64))
    assert e.value.status == 1
    with pytest.raises(ls.LsortError) as e:        # first offset not 0
        S.sort_segments_device_(t, dev(np.array([3, 16], dtype=np.int64), np.int64))
    assert e.value.status == 1
    a = np.random.default_rng(8).normal(size=16)
    t2 = torch.from_numpy(a.copy()).to("cuda:0")
    S.sort_segments_device_(t2, dev(np.array([0, 16], dtype=np.int64), np.int64))
    torch.cuda.synchronize()
    assert np.array_equal(words_of(t2), expected_sorted(a))
