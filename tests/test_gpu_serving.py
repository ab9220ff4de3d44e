"""The continuous-batching server: a request's result is the same alone and in a
mix of concurrent requests of uneven size and k (the query key is the index
within the request), admission limits are respected, and bad requests are
rejected before anything runs."""
import threading

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare, dev, oracle_kwargs, say, to_device_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")


@pytest.fixture(scope="module")
def served():
    X = synth.mixture_small(4000, 64, 16, 0.3, 101)
    ox = oracle.build_index(X, deg=32, S=2, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    return X, ox, gx


def direct(gx, Q, k, itopk, T, opts):
    ids, dists = gx.search(dev(Q), k, itopk, T, opts,
                           qkeys=torch.arange(len(Q), dtype=torch.int64).cuda())
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), dists.cpu().numpy()


def oracle_of(ox, Q, k, itopk, T, opts):
    """The CPU oracle's result for one request: query keys are the rows' indices in the request."""
    o = oracle.search(ox, Q, qkeys=np.arange(len(Q), dtype=np.uint64), **oracle_kwargs(k, itopk, T, opts))
    return o


def test_alone_equals_in_mix(served):
    X, ox, gx = served
    opts = miann.SearchOptions(entry="ghost_graph", dgs=True)
    rng = np.random.default_rng(5)
    A = synth.mixture_small(37, 64, 16, 0.3, 102)
    srv = miann.Server(gx, num_streams=4, max_batch_queries=2048)
    tA = srv.submit(A, 10, 64, 60, opts)
    ia, da, _ = srv.wait(tA, len(A), 10)
    ref_i, ref_d = direct(gx, A, 10, 64, 60, opts)
    assert np.array_equal(ia, ref_i) and np.array_equal(da, ref_d)
    # the same request inside a mix of uneven requests submitted from two threads
    reqs = []
    for j in range(40):
        n = int(min(1024, np.floor(np.exp(rng.uniform(0, np.log(1025))))))
        k = int(rng.choice([10, 32]))
        reqs.append((synth.mixture_small(max(1, n), 64, 16, 0.3, 200 + j), k))
    tickets = [None] * len(reqs)
    mid = []

    def submit(lo, hi):
        for j in range(lo, hi):
            tickets[j] = srv.submit(reqs[j][0], reqs[j][1], 64, 60, opts)
            if j == 20:
                mid.append(srv.submit(A, 10, 64, 60, opts))

    th = [threading.Thread(target=submit, args=(0, 20)), threading.Thread(target=submit, args=(20, 40))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    ib, db, _ = srv.wait(mid[0], len(A), 10)
    assert np.array_equal(ib, ia) and np.array_equal(db, da)
    lats = []
    for j, (Qj, k) in enumerate(reqs):
        ij, dj, lat = srv.wait(tickets[j], len(Qj), k)
        lats.append(lat)
        ri, rd = direct(gx, Qj, k, 64, 60, opts)
        assert np.array_equal(ij, ri) and np.array_equal(dj, rd), j
        # and the CPU oracle's result for the request on its own
        compare((ij, dj, None), oracle_of(ox, Qj, k, 64, 60, opts), check_counters=False, label=f"served {j}")
    st = srv.stats()
    say(f"  batches {st['batches']} for {st['requests_done']} requests; p50 {np.percentile(lats, 50):.2f} ms "
        f"p99 {np.percentile(lats, 99):.2f} ms")
    assert st["requests_done"] == len(reqs) + 2
    srv.close()


def test_admission_limits_queue_requests(served):
    X, ox, gx = served
    opts = miann.SearchOptions(entry="ghost_graph")
    srv = miann.Server(gx, num_streams=3, max_batch_queries=64, max_inflight_queries=96,
                       memory_budget_bytes=200_000)
    Qs = [synth.mixture_small(n, 64, 16, 0.3, 300 + n) for n in (60, 50, 40, 30, 64, 1, 2, 33)]
    ts = [srv.submit(Q, 10, 32, 30, opts) for Q in Qs]
    for t, Q in zip(ts, Qs):
        ids, _, _ = srv.wait(t, len(Q), 10)
        ri, _ = direct(gx, Q, 10, 32, 30, opts)
        assert np.array_equal(ids, ri)
    st = srv.stats()
    assert st["peak_inflight_queries"] <= 96 and st["peak_inflight_bytes"] <= 200_000
    with pytest.raises(miann.MiannError):
        srv.submit(synth.mixture_small(65, 64, 16, 0.3, 1), 10, 32, 30, opts)  # larger than one batch
    with pytest.raises(miann.MiannError):
        srv.submit(Qs[0], 40, 32, 30, opts)  # k > itopk
    srv.close()


def test_u8_degree64_dense_entry_mix():
    """The serving form of the benchmark: uint8 rows, degree-64 graph, dense ghost entry with the direction
    filter, requests of 1..1,024 queries with k in {10, 100} on four server streams (each stream with its own
    kept scratch). Every served result equals the direct search of the same request and the CPU oracle's,
    bit for bit (exact int32 distances)."""
    say("serving u8 degree 64 dense entry, k in {10, 100}")
    X = synth.to_u8(synth.mixture_small(3000, 128, 8, 0.3, 111))
    ox = oracle.build_index(X, deg=64, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    opts = miann.SearchOptions(entry="ghost_dense", dgs=True)
    setting = {10: (64, 32), 100: (128, 48)}
    rng = np.random.default_rng(17)
    reqs = []
    for j in range(24):
        n = int(min(1024, np.floor(np.exp(rng.uniform(0, np.log(1025))))))
        reqs.append((synth.to_u8(synth.mixture_small(max(1, n), 128, 8, 0.3, 400 + j)), int(rng.choice([10, 100]))))
    srv = miann.Server(gx, num_streams=4, max_batch_queries=4096)
    tickets = [srv.submit(Qj, k, *setting[k], opts) for Qj, k in reqs]
    for j, (Qj, k) in enumerate(reqs):
        ij, dj, _ = srv.wait(tickets[j], len(Qj), k)
        ri, rd = direct(gx, Qj, k, *setting[k], opts)
        assert np.array_equal(ij, ri) and np.array_equal(dj, rd), j
        frac = compare((ij, dj, None), oracle_of(ox, Qj, k, *setting[k], opts), min_frac=1.0, check_counters=False,
                       label=f"u8 served {j} k={k} n={len(Qj)}")
        assert frac == 1.0
    st = srv.stats()
    assert st["requests_done"] == len(reqs)
    srv.close()


def test_warm_and_replay_trace(served):
    """The native load generator: requests arrive at their scheduled times from a thread of the library, every
    one completes, latencies run from the scheduled arrival, and a request replayed this way returns what the
    direct search returns (checked by submitting it again after the replay)."""
    X, ox, gx = served
    opts = miann.SearchOptions(entry="ghost_dense", dgs=True)
    srv = miann.Server(gx, num_streams=4, max_batch_queries=2048)
    srv.warm(512, 10, 64, 40, opts)
    srv.warm(512, 32, 64, 40, opts)
    rng = np.random.default_rng(23)
    n_req = 200
    sizes = np.minimum(256, np.floor(np.exp(rng.uniform(0, np.log(257), n_req)))).astype(np.int64)
    pool = synth.mixture_small(int(sizes.sum()), 64, 16, 0.3, 131)
    off = np.concatenate([[0], np.cumsum(sizes)])
    ks = rng.choice([10, 32], n_req).astype(np.int32)
    arrivals = np.cumsum(rng.exponential(0.002, n_req))
    lat, wall = srv.replay(pool, off[:-1], sizes, ks, np.full(n_req, 64), np.full(n_req, 40), arrivals, opts)
    say(f"  replay of {n_req} requests over {arrivals[-1]:.3f} s: wall {wall:.3f} s, p50 {np.percentile(lat, 50):.2f} ms"
        f" p99 {np.percentile(lat, 99):.2f} ms")
    assert np.all(lat > 0) and wall >= arrivals[-1]
    st = srv.stats()
    assert st["requests_done"] >= n_req
    j = int(np.argmax(sizes))
    t = srv.submit(pool[off[j]:off[j + 1]], int(ks[j]), 64, 40, opts)
    ij, dj, _ = srv.wait(t)
    ri, rd = direct(gx, pool[off[j]:off[j + 1]], int(ks[j]), 64, 40, opts)
    assert np.array_equal(ij, ri) and np.array_equal(dj, rd)
    srv.close()
