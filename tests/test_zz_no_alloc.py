"""The no-allocation sort (ls_sort_noalloc) through the C ABI: on two calls in
a row, the second with a smaller input, each output equals the bits of the
ordinary entry point (ls_sort_f64 / ls_sort_u64) on the same keys and the
plain definition of the result; the device's free memory does not move during
the calls; sizes beyond the limit are rejected before any work."""
import numpy as np
import pytest

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


def cases():
    r = np.random.default_rng(2107)
    specials = r.choice(np.concatenate([SPECIAL_F64, [np.nan, -np.nan]]), size=300_001)
    return [
        ("mixed_u64", W.mixed_u64(ls.NOALLOC_MAX_KEYS, seed=31), W.mixed_u64(300_001, seed=32)),
        ("uniform_f64", W.uniform_1e9grid(ls.NOALLOC_MAX_KEYS, seed=33), specials),
        ("zipf_f64", W.zipf_lognormal(1_000_000, seed=34, distinct=20_000), r.normal(size=4_097)),
    ]


@pytest.mark.parametrize("name,first,second", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_noalloc_equals_plain_on_two_calls(S, name, first, second):
    for keys in (first, second):       # the second call is smaller
        print("noalloc case %s n=%d" % (name, keys.size), flush=True)
        plain = to_dev(keys)
        S.sort_(plain)
        torch.cuda.synchronize()
        t = to_dev(keys)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(0)[0]
        S.sort_noalloc_(t)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(0)[0]
        got = words_of(t)
        assert np.array_equal(got, words_of(plain))
        assert np.array_equal(got, expected_sorted(keys))
        assert free1 == free0


def test_noalloc_small_and_parameter_sweep(S):
    r = np.random.default_rng(5)
    for n in (0, 1, 2, 3, 1000, 8192, 8193, 65_537):
        keys = r.lognormal(0, 2, size=n)
        t = to_dev(keys)
        S.sort_noalloc_(t, ls.params(fanout=256, base_threshold=1024, tile=2048))
        torch.cuda.synchronize()
        assert np.array_equal(words_of(t), expected_sorted(keys))


def test_noalloc_rejects_beyond_the_limit(S):
    t = torch.zeros(ls.NOALLOC_MAX_KEYS + 1, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ls.LsortError) as e:
        S.sort_noalloc_(t)
    assert e.value.status == 4
    assert int(t.abs().sum()) == 0
    with pytest.raises(ls.LsortError) as e:
        S.sort_noalloc_(t[:1000], ls.params(flags=ls.FLAG_PROFILE))
    assert e.value.status == 4
