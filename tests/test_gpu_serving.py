"""GPU tests of the serving loop: every result equals the client's next
numbers from the oracle, results are identical alone and in the mix
(tolerance 0), admission respects the HBM budget and per-client order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def mods(torch):
    from paper_1112_5239_amd import generator, serving, workloads
    return generator, serving, workloads


_HIP = None


def _copy_result(torch, c):
    """Device result of a completion -> host uint32 array (hipMemcpy D2H)."""
    import ctypes
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    n = int(c.length)
    host = np.empty(n, dtype=np.uint32)
    assert _HIP.hipMemcpy(host.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(c.out), n * 4, 2) == 0
    return host


def _small_trace(seed, n_req=300, n_clients=40, rate=2000.0, max_numbers=1 << 20):
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, n_req)) * 1e9
    client = rng.integers(0, n_clients, n_req).astype(np.uint32)
    u = rng.random(n_req)
    length = np.maximum(1, np.floor(np.power(max_numbers, u))).astype(np.uint64)
    return arrival.astype(np.uint64), client, length


def test_replay_matches_oracle_per_client(orc, torch, mods):
    G, S, _ = mods
    arrival, client, length = _small_trace(1)
    n_clients = 40
    gen = G.Generator(n_clients, "v0", seed=4)
    srv = S.Server(gen, n_gpu_streams=3, budget_bytes=1 << 30)
    try:
        res = srv.replay(arrival, client, length, release_results=False)
        assert {int(res[i].status) for i in range(len(arrival))} == {0}
        st = orc.seed(0, 4, 0, n_clients)
        per_client = {}
        for i in range(len(arrival)):
            per_client.setdefault(int(client[i]), []).append(i)
        for c, idx in per_client.items():
            total = int(sum(int(length[i]) for i in idx))
            want, _ = orc.generate(0, st[c:c + 1], total)
            pos = 0
            for i in idx:                       # the client's requests in submission order
                got = _copy_result(torch, res[i])
                L = int(length[i])
                assert np.array_equal(got, want[0, pos:pos + L]), f"client {c} request {i}"
                pos += L
        assert np.array_equal(gen.get_state(), st)
        for i in range(len(arrival)):
            srv.release(res[i].out)
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.close()
        gen.close()


def test_alone_and_in_the_mix_identical(torch, mods):
    G, S, _ = mods
    arrival, client, length = _small_trace(2, n_req=200, n_clients=16)
    target = int(client[0])
    # in the mix
    gen = G.Generator(16, "v0", seed=9)
    srv = S.Server(gen, n_gpu_streams=2, budget_bytes=1 << 30)
    try:
        res = srv.replay(arrival, client, length, release_results=False)
        mixed = [_copy_result(torch, res[i]) for i in range(len(arrival)) if int(client[i]) == target]
    finally:
        srv.close()
        gen.close()
    # alone: only the target client's requests, same times
    sel = client == target
    gen = G.Generator(16, "v0", seed=9)
    srv = S.Server(gen, n_gpu_streams=1, budget_bytes=1 << 30)
    try:
        res = srv.replay(arrival[sel], client[sel], length[sel], release_results=False)
        alone = [_copy_result(torch, res[i]) for i in range(int(sel.sum()))]
    finally:
        srv.close()
        gen.close()
    assert len(mixed) == len(alone) > 1
    for a, b in zip(mixed, alone):
        assert np.array_equal(a, b)


def test_budget_admission_and_client_order(orc, torch, mods):
    G, S, _ = mods
    gen = G.Generator(8, "v0", seed=5)
    budget = 1 << 20                              # 1 MiB of results
    srv = S.Server(gen, n_gpu_streams=2, budget_bytes=budget)
    try:
        n = 96 << 10                              # 384 KiB per request: two fit, not three
        for tag, c in enumerate([0, 1, 2, 0, 3]):
            srv.submit(c, n, tag)
        done = {}
        seen_max = 0
        for _ in range(2000):
            for c in srv.poll():
                done[int(c.tag)] = c
            seen_max = max(seen_max, srv.stats()["bytes_in_use"])
            if len(done) >= 2:
                break
        st = srv.stats()
        assert st["bytes_in_use"] <= budget and seen_max <= budget
        assert len(done) + st["in_flight"] <= 2     # the third result does not fit
        assert st["waiting"] >= 3
        # releasing results lets the rest in, in each client's order
        results = {}
        for _ in range(20000):
            for t, c in list(done.items()):
                results[t] = _copy_result(torch, c)
                srv.release(c.out)
                del done[t]
            for c in srv.poll():
                done[int(c.tag)] = c
            if len(results) + len(done) == 5 and not srv.stats()["in_flight"]:
                break
        for t, c in list(done.items()):
            results[t] = _copy_result(torch, c)
            srv.release(c.out)
        assert sorted(results) == [0, 1, 2, 3, 4]
        ref = orc.seed(0, 5, 0, 8)
        want0, _ = orc.generate(0, ref[0:1], 2 * n)
        assert np.array_equal(results[0], want0[0, :n])
        assert np.array_equal(results[3], want0[0, n:])        # client 0's second request
        for t, c in ((1, 1), (2, 2), (4, 3)):
            w, _ = orc.generate(0, ref[c:c + 1], n)
            assert np.array_equal(results[t], w[0])
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.close()
        gen.close()


def test_submit_rejects_bad_requests(mods):
    G, S, _ = mods
    from paper_1112_5239_amd import CprngError
    gen = G.Generator(4, "v0", seed=1)
    srv = S.Server(gen, budget_bytes=1 << 20)
    try:
        with pytest.raises(CprngError):
            srv.submit(4, 10, 0)                  # client out of range
        with pytest.raises(CprngError):
            srv.submit(0, 0, 0)                   # empty
        with pytest.raises(CprngError):
            srv.submit(0, (1 << 20) // 4 + 1, 0)  # larger than the budget
    finally:
        srv.close()
        gen.close()
    g1 = G.Generator(64, "v2", seed=1)
    try:
        with pytest.raises(CprngError):
            S.Server(g1)
    finally:
        g1.close()


def test_serving_workload_short_sampled(orc, torch, mods):
    # The benchmark's trace shape (1 KiB..256 MiB, 10,000 clients), 0.5 s of
    # arrivals, results kept for a sample of clients.
    G, S, W = mods
    arrival, client, length = W.serving_trace(duration_s=0.5)
    gen = G.Generator(10000, "v0", seed=4)
    srv = S.Server(gen, n_gpu_streams=2, budget_bytes=64 << 30)
    try:
        res = srv.replay(arrival, client, length, release_results=False)
        n = len(arrival)
        assert {int(res[i].status) for i in range(n)} == {0}
        lat = np.array([res[i].t_done_ns - res[i].t_submit_ns for i in range(n)])
        assert (lat > 0).all()
        st = orc.seed(0, 4, 0, 10000)
        pick = np.unique(client)[:50]
        for c in pick:
            idx = [i for i in range(n) if int(client[i]) == int(c)]
            total = int(sum(int(length[i]) for i in idx))
            want, _ = orc.generate(0, st[int(c):int(c) + 1].copy(), total)
            pos = 0
            for i in idx:
                L = int(length[i])
                assert np.array_equal(_copy_result(torch, res[i]), want[0, pos:pos + L]), f"client {c}"
                pos += L
        for i in range(n):
            srv.release(res[i].out)
    finally:
        srv.close()
        gen.close()


def test_serving_trace_seconds_checked(orc, torch, mods):
    # The benchmark's serving leg (serving.run_trace) on 3 s of its trace,
    # with every result of 20 sampled clients kept and compared with the
    # oracle generating each of those clients' streams alone; every other
    # result is released as it completes.
    G, S, W = mods
    st = orc.seed(0, 4, 0, 10000)
    seen = []

    def check(c, results):
        total = sum(r.size for r in results)
        want, _ = orc.generate(0, st[c:c + 1].copy(), total)
        pos = 0
        for k, r in enumerate(results):
            assert np.array_equal(r, want[0, pos:pos + r.size]), f"client {c} request {k}"
            pos += r.size
        seen.append(c)

    summary = S.run_trace(3.0, check_clients=20, oracle_check=check)
    assert summary["statuses"] == [0]
    assert summary["clients_checked"] == len(seen) == 20
    assert summary["latency_ms"]["p50"] > 0
