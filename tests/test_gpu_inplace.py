"""In-place partition rounds (LS_FLAG_INPLACE: Alg. 1 with fragments written
back into the input, then Defragment as a block permutation) through the C
ABI.  Bar: bit-exact against the definition of the result and the CPU
oracle, exactly as the out-of-place sort; the extra device memory stays a
small fraction of the keys' bytes."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import expected_sorted, raw_words
from tests.test_gpu_parity import NAMES, inputs

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


def sort_inplace(S, a, **kw):
    t = to_dev(a)
    S.sort_(t, ls.params(flags=ls.FLAG_INPLACE | kw.pop("flags", 0), **kw))
    torch.cuda.synchronize()
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def test_inplace_small_first(S):
    a = inputs("uniform", 100_003, 5)
    print("inplace uniform n=%d" % a.size, flush=True)
    assert np.array_equal(sort_inplace(S, a), expected_sorted(a))


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 4095, 4097, 100_003, 1_000_000])
def test_inplace_matches_definition_and_oracle(S, name, n):
    a = inputs(name, n, n + 29)
    got = sort_inplace(S, a)
    assert np.array_equal(got, expected_sorted(a))
    if 0 < n <= 100_003:
        s, _ = oracle.sort(a, s_max=4096)
        assert np.array_equal(got, raw_words(s))


@pytest.mark.parametrize("kw", [dict(fanout=2), dict(fanout=16, leaves=8), dict(fanout=64),
                                dict(fanout=1024), dict(base_threshold=2), dict(base_threshold=64, fanout=8),
                                dict(sample_cap=100), dict(leaves=1), dict(flags=ls.FLAG_NONMONOTONE)])
@pytest.mark.parametrize("name", ["uniform", "zipf", "mixed_u64", "twovalues"])
def test_inplace_parameters(S, kw, name):
    a = inputs(name, 300_001, 41)
    assert np.array_equal(sort_inplace(S, a, **dict(kw)), expected_sorted(a))


def test_inplace_recursion_and_fallbacks(S):
    # duplicate-heavy ranges recurse below level 1 with local models and the
    # highest-differing-bit split
    a = W.mixed_u64(3_000_000, seed=44)
    assert np.array_equal(sort_inplace(S, a), expected_sorted(a))
    b = np.repeat(np.array([2.0 ** 62 + k for k in range(5)], dtype=np.uint64), 40_000)
    np.random.default_rng(3).shuffle(b)
    assert np.array_equal(sort_inplace(S, b), expected_sorted(b))


def test_inplace_segments(S):
    spec = W.segment_spec(count=60, seed=45, hi=1 << 18)
    keys = W.segments(spec)
    off = spec.offsets
    t = to_dev(keys)
    S.sort_segments_(t, off, p=ls.params(flags=ls.FLAG_INPLACE))
    torch.cuda.synchronize()
    got = t.view(torch.int64).cpu().numpy().view(np.uint64)
    for i in range(off.size - 1):
        lo, hi = int(off[i]), int(off[i + 1])
        assert np.array_equal(got[lo:hi], expected_sorted(keys[lo:hi])), i


def test_inplace_extra_memory_is_small():
    # a fresh context: the device memory its work buffers hold after an
    # in-place sort of 2^27 keys (round tables, block tags and flags, side
    # buffer, overflow blocks, models, lists) against the 1 GB of keys; the
    # out-of-place sort holds a whole key-sized scratch buffer besides.  The
    # device's free memory drops by that plus what the HIP runtime allocates
    # for the new context's streams (about 14 MB measured)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 1 << 27
    a = W.mixed_u64(n, seed=46)
    t = to_dev(a)
    torch.cuda.synchronize()
    s = ls.Sorter(0)
    try:
        free0 = torch.cuda.mem_get_info(0)[0]
        s.sort_(t, ls.params(flags=ls.FLAG_INPLACE))
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info(0)[0]
        held = s.device_bytes()
        print("in-place n=2^27: context holds %.1f MB, device free memory -%.1f MB" % (held / 1e6, used / 1e6))
    finally:
        s.close()
    assert held <= 0.10 * n * 8, held
    assert used <= 0.10 * n * 8 + (32 << 20), used
    got = t.view(torch.int64).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, expected_sorted(a))
