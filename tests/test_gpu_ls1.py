"""LearnedSort 1.0's spill bucket on the GPU (ls_sort_ls1, the ablation of
Sec. 2 / Fig. 1 / Sec. 3) through the C ABI.  Bar: bit-exact against the
definition of the result (the sorted order is unique) and the CPU oracle,
whatever spills; the spill bucket fills with repeated keys."""
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


def sort_ls1(S, a, slack=0.1, **kw):
    t = to_dev(a)
    st = S.sort_ls1_(t, slack=slack, p=ls.params(**kw) if kw else None)
    torch.cuda.synchronize()
    return t.view(torch.int64).cpu().numpy().view(np.uint64), st


def test_ls1_small_first(S):
    a = inputs("uniform", 100_003, 5)
    print("ls1 uniform n=%d" % a.size, flush=True)
    got, st = sort_ls1(S, a)
    assert np.array_equal(got, expected_sorted(a))


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4097, 100_003, 1_000_000])
def test_ls1_matches_definition_and_oracle(S, name, n):
    a = inputs(name, n, n + 31)
    got, st = sort_ls1(S, a)
    assert np.array_equal(got, expected_sorted(a))
    if 0 < n <= 100_003:
        s, _ = oracle.sort(a, s_max=4096)
        assert np.array_equal(got, raw_words(s))
    if n > 1:
        assert st["spilled"] <= n and st["capacity"] >= 1


@pytest.mark.parametrize("slack", [0.0, 0.1, 1.0])
@pytest.mark.parametrize("kw", [dict(), dict(fanout=2), dict(fanout=64, leaves=16), dict(fanout=1000, leaves=1000)])
def test_ls1_parameters(S, slack, kw):
    a = inputs("zipf", 300_001, 43)
    got, st = sort_ls1(S, a, slack=slack, **kw)
    assert np.array_equal(got, expected_sorted(a))
    f = kw.get("fanout", 1024)
    assert st["fanout"] == f
    assert st["capacity"] == int(np.ceil(a.size * (1 + slack) / f))


@pytest.mark.parametrize("fam", ["uniform", "exponential", "zipf0.90"])
def test_spill_is_the_overflow_of_the_level0_buckets(S, fam):
    # LS1's spill bucket holds exactly what the fixed capacities cannot:
    # sum over buckets of max(0, size - capacity), the sizes from the
    # oracle's level-0 stage (same model, same buckets).  Distinct keys
    # spread over the buckets and barely spill; every copy of a repeated key
    # lands in one bucket and overflows it (Sec. 3)
    n = 1 << 21
    a = W.paper_family_large(fam, n, seed=3)
    got, st = sort_ls1(S, a, slack=0.1)
    assert np.array_equal(got, expected_sorted(a))
    sizes = oracle.stage_level0(a, fanout=1024, leaves=1024)["sb"].astype(np.int64)
    cap = int(np.ceil(n * 1.1 / 1024))
    want = int(np.maximum(sizes - cap, 0).sum())
    print("%s: spilled %d of %d (%.1f%%)" % (fam, st["spilled"], n, 100.0 * st["spilled"] / n))
    assert st["capacity"] == cap and st["spilled"] == want
    if fam == "zipf0.90":
        assert st["spilled"] > 0.1 * n
    else:
        assert st["spilled"] < 0.05 * n


def test_ls1_rejects_bad_arguments(S):
    t = torch.zeros(100, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ls.LsortError):
        S.sort_ls1_(t, slack=-1.0)
    with pytest.raises(ls.LsortError) as e:
        S.sort_ls1_(t, p=ls.params(fanout=4096))     # its LDS does not fit one workgroup
    assert e.value.status == 4
