"""The continuous-batching server: every request's result is the same alone
and in the mix (bit-exact), admission respects the HBM budget, requests that
arrive while batches run are picked up, and batches replayed from captured
HIP graphs give the same bits."""
import threading

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
    t = torch.from_numpy(raw_words(a).view(np.int64).copy()).to("cuda:0")
    return t.view(torch.float64) if a.dtype == np.float64 else t


def words(t) -> np.ndarray:
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def request_inputs(count, seed, hi):
    spec = W.request_spec(count=count, seed=seed, lo=1, hi=hi)
    return [W.request_keys(spec, i) for i in range(count)]


def test_same_result_alone_and_in_the_mix(S):
    reqs = request_inputs(48, seed=31, hi=1 << 21)
    alone = []
    for a in reqs:
        t = upload(a)
        S.sort_(t)
        alone.append(t)
    mixed = [upload(a) for a in reqs]
    torch.cuda.synchronize()
    srv = ls.Server(0, hbm_budget=8 << 30, max_inflight=3)
    try:
        tickets = [srv.submit(t) for t in mixed]
        lat = [srv.wait(tk) for tk in tickets]
        st = srv.stats()
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert all(x >= 0 for x in lat)
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["batches"] < len(reqs)            # requests were batched
    for a, t1, t2 in zip(reqs, alone, mixed):
        assert torch.equal(t1.view(torch.int64), t2.view(torch.int64))
    for i in (0, 7, 21, 47):
        assert np.array_equal(words(mixed[i]), expected_sorted(reqs[i]))


def batch_bound(S, n):
    # the server's bound on what a batch of n keys adds to a context
    return int(S.workspace_size(n) * 1.5) + (8 << 20)


def test_budget_bounds_device_memory(S):
    # The device's free memory is polled while the server runs: what the
    # server's contexts allocate stays within the budget (whose other part is
    # the keys in flight, allocated here beforehand), up to what the HIP
    # runtime takes for the workers' streams.  The budget holds about one
    # batch of the largest requests at a time, so workers must free the
    # buffers they keep from earlier batches for the next one to run.
    reqs = request_inputs(40, seed=32, hi=1 << 22)
    ts = [upload(a) for a in reqs]
    torch.cuda.synchronize()
    biggest = max(a.size for a in reqs)
    one = biggest * 8 + batch_bound(S, biggest)
    budget = int(one * 1.3)
    workers = 3
    free0 = torch.cuda.mem_get_info(0)[0]
    srv = ls.Server(0, hbm_budget=budget, max_inflight=workers)
    peak_used = 0
    try:
        too_big = torch.empty(budget // 8, dtype=torch.float64, device="cuda:0")
        with pytest.raises(ls.LsortError) as e:
            srv.submit(too_big)
        assert e.value.status == 5
        del too_big
        torch.cuda.empty_cache()
        free0 = min(free0, torch.cuda.mem_get_info(0)[0])
        tickets = [srv.submit(t) for t in ts]
        for tk in tickets:
            while True:
                try:
                    srv.wait(tk, timeout_ms=1)
                    break
                except ls.LsortError as e:
                    if e.status != 6:
                        raise
                peak_used = max(peak_used, free0 - torch.cuda.mem_get_info(0)[0])
        st = srv.stats()
        with pytest.raises(ls.LsortError) as e:
            srv.wait(10 ** 9)
        assert e.value.status == 7
    finally:
        srv.close()
    print("budget %.1f MB, peak accounted %.1f MB, peak device use of the server %.1f MB, batches %d" %
          (budget / 1e6, st["peak_bytes"] / 1e6, peak_used / 1e6, st["batches"]))
    assert st["completed"] == len(reqs) and st["queued"] == 0
    assert 0 < st["peak_bytes"] <= budget
    assert peak_used <= budget + workers * (16 << 20), peak_used
    for a, t in zip(reqs, ts):
        assert np.array_equal(words(t), expected_sorted(a))


def test_concurrent_submitters_while_batches_run():
    reqs = request_inputs(64, seed=33, hi=1 << 22)
    ts = [upload(a) for a in reqs]
    torch.cuda.synchronize()
    srv = ls.Server(0, hbm_budget=4 << 30, max_inflight=2)
    tickets = [None] * len(ts)

    def submitter(k):
        for i in range(k, len(ts), 4):
            tickets[i] = srv.submit(ts[i])

    try:
        th = [threading.Thread(target=submitter, args=(k,)) for k in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for tk in tickets:
            srv.wait(tk)
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(ts)
    for a, t in zip(reqs, ts):
        assert np.array_equal(words(t), expected_sorted(a))


def test_graph_batches_in_the_server(S):
    spec = W.request_spec(count=40, seed=34, lo=1, hi=1 << 23)
    # batches of up to 2^22 keys replay graphs captured by two workers at
    # once; larger batches run host-driven in between on the same contexts
    reqs = [W.request_keys(spec, i) for i in range(40)]
    ts = [upload(a) for a in reqs]
    torch.cuda.synchronize()
    print("server+graph: %d requests, %d keys" % (len(reqs), sum(a.size for a in reqs)), flush=True)
    srv = ls.Server(0, hbm_budget=4 << 30, max_inflight=2, p=ls.params(flags=ls.FLAG_GRAPH))
    try:
        tickets = [srv.submit(t) for t in ts]
        for tk in tickets:
            srv.wait(tk)
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(ts)
    for a, t in zip(reqs, ts):
        assert np.array_equal(words(t), expected_sorted(a))
