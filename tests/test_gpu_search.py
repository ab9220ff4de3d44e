"""GPU parity of the HIP search path against the CPU oracle.

Every case imports an oracle-built index (graphs, shard maps, ghost shards)
into the library, so search parity is tested independently of build parity,
and runs the same queries with the same parameters on both sides. The bar:
the id lists match on >= 99.9% of queries (float distances within 1e-5
relative, uint8 distances bit-exact), and the per-query expansion, iteration,
skipped-slot and rerank counts agree.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare, dev, ghost_entry, run_both, say, to_device_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")

K = 10


def mix(n, d, C, sigma, seed):
    return synth.mixture_small(n, d, C, sigma, seed)


@pytest.fixture(scope="module")
def small():
    """N = 3,000, d = 128, 8 components; ghost sample of 5% with a degree-16 ghost graph."""
    X = mix(3000, 128, 8, 0.3, 11)
    Q = mix(300, 128, 8, 0.3, 12)
    ox = oracle.build_index(X, deg=32, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    return X, Q, ox, gx


CASES = [
    ("plain", 64, 80, dict()),
    ("dgs", 64, 80, dict(dgs=True)),
    ("dgs_r2", 64, 60, dict(dgs=True, search_width=2)),
    ("r2", 64, 60, dict(search_width=2)),
    ("ghost_graph", 64, 80, dict(entry="ghost_graph")),
    ("ghost_graph_dgs", 64, 80, dict(entry="ghost_graph", dgs=True, ghost_iters=5, t_seeds=16)),
    ("ghost_dense", 64, 80, dict(entry="ghost_dense")),
    ("random_discard", 64, 80, dict(dgs=True, random_discard=True)),
    ("stop_on_no_change", 64, 200, dict(stop_on_no_change=True)),
    ("n_init_300_small_hash", 64, 80, dict(n_init=300, hash_log2=8)),
    ("itopk_256", 256, 300, dict(dgs=True, cooldown=0.5)),
    ("itopk_k", 10, 40, dict()),
    ("T0", 64, 0, dict(n_init=100)),
    ("discard_07", 64, 80, dict(dgs=True, discard=0.7, cooldown=0.1)),
    ("discard_0625_c0_r2", 32, 8, dict(dgs=True, discard=0.625, cooldown=0.0, search_width=2)),
    ("discard_075_c0_r2", 32, 9, dict(dgs=True, discard=0.75, cooldown=0.0, search_width=2)),
    ("dgs_threshold_040", 64, 80, dict(dgs=True, dgs_threshold=0.4)),
    ("dgs_threshold_035_r2", 64, 60, dict(dgs=True, dgs_threshold=0.35, search_width=2)),
]


@pytest.mark.parametrize("name,itopk,T,kw", CASES, ids=[c[0] for c in CASES])
def test_search_parity_small(small, name, itopk, T, kw):
    X, Q, ox, gx = small
    say(f"case {name}: nq={len(Q)} itopk={itopk} T={T} {kw}")
    opts = miann.SearchOptions(**kw)
    g, o = run_both(ox, gx, Q, min(K, itopk), itopk, T, opts)
    compare(g, o, label=name, ndist_check=not ghost_entry(opts))


@pytest.mark.parametrize("d", [16, 100, 200])
def test_search_parity_odd_dims(d):
    say(f"odd dims d={d}")
    X = mix(1500, d, 5, 0.3, 21)
    Q = mix(100, d, 5, 0.3, 22)
    ox = oracle.build_index(X, deg=16, dgs=True, ghost_R=100, deg_g=8)
    gx = to_device_index(ox)
    for kw in (dict(), dict(dgs=True, entry="ghost_graph"), dict(entry="ghost_dense", search_width=4)):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, 48, 60, opts)
        compare(g, o, label=f"d{d}-{kw}", ndist_check=not ghost_entry(opts))


def test_dense_entry_equidistant_ghosts():
    """Dense entry when every ghost is equidistant from the query: sign vectors in {-1, 1}^32 (all of squared norm
    32 exactly) and queries at the origin. Every ghost passes the GEMM-form bound, so each list is longer than the
    rescoring capacity and the kernel falls back to its exact scan; the seeds must still be the exact top-t by
    (dist, id). Half-scaled copies of data points as queries exercise the ordinary path on the same index."""
    say("dense entry, equidistant ghosts")
    rng = np.random.default_rng(61)
    d = 32
    X = rng.choice(np.array([-1.0, 1.0], dtype=np.float32), size=(2000, d))
    Q = np.concatenate([np.zeros((16, d), np.float32), 0.5 * X[:16]]).astype(np.float32)
    ox = oracle.build_index(X, deg=16, dgs=True, ghost_R=400, deg_g=8)
    gx = to_device_index(ox)
    for kw in (dict(entry="ghost_dense"), dict(entry="ghost_dense", dgs=True, t_seeds=48),
               dict(entry="ghost_dense", t_seeds=8), dict(entry="ghost_dense", dgs=True, t_seeds=20)):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, 48, 20, opts)
        compare(g, o, label=f"signs-{kw}", ndist_check=False)


@pytest.mark.parametrize("t,n_near", [(8, 30), (20, 30), (8, 100)])
def test_dense_entry_near_ties_inside_the_window(t, n_near):
    """Near ties the GEMM form cannot separate: around each query, n_near ghosts at distances 1 + k 1e-6 (a spacing
    far below the GEMM form's error bound, but resolved by the exact distance), the other ghosts at distance 2 or
    more. With every node a ghost and T = 0, the result is the exact top-k of the t seeds, so the seeds must be
    the exact top-t of the n_near (the window holds all of them and is rescored exactly). 30 near ghosts fit one
    8-lane team's list; 100 take the per-wave path for longer lists."""
    rng = np.random.default_rng(62)
    d, n_q = 64, 8
    Q = (10.0 * rng.standard_normal((n_q, d)) / np.sqrt(d)).astype(np.float32)
    rows = []
    for q in Q:
        u = rng.standard_normal((n_near, d))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = np.sqrt(1.0 + 1e-6 * rng.permutation(n_near))[:, None]
        rows.append(q + u * r)
        v = rng.standard_normal((30, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        rows.append(q + v * (2.0 + rng.random((30, 1))))
    X = np.concatenate(rows).astype(np.float32)
    ox = oracle.build_index(X, deg=16, dgs=False, ghost_R=len(X), deg_g=16)
    gx = to_device_index(ox, dgs=False)
    opts = miann.SearchOptions(entry="ghost_dense", t_seeds=t)
    g, o = run_both(ox, gx, Q, t, 32, 0, opts)
    compare(g, o, min_frac=1.0, label=f"near-ties-t{t}-n{n_near}", ndist_check=False)


@pytest.mark.parametrize("S", [2, 3])
def test_path_extension_parity(S):
    """Path extension across S resident shards (Sec. 3.1.2) and naive sharding."""
    say(f"shards S={S}")
    X = mix(3000, 96, 8, 0.25, 31)
    Q = mix(200, 96, 8, 0.25, 32)
    ox = oracle.build_index(X, deg=32, S=S, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    for kw in (dict(), dict(dgs=True, entry="ghost_graph"), dict(ppe=False, entry="ghost_dense"),
               dict(forward_f=4, dgs=True), dict(ppe=False),
               dict(entry="ghost_dense", dgs=True, ghost_every_stage=True),
               dict(entry="ghost_graph", ghost_every_stage=True, search_width=2)):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, 64, 50, opts)
        compare(g, o, label=f"S{S}-{kw}", ndist_check=not ghost_entry(opts))


@pytest.mark.parametrize("discard,T", [(0.5, 6), (0.5, 7), (0.625, 7), (0.625, 8), (0.75, 9)])
def test_sharded_dense_every_stage_no_cooldown(discard, T):
    """The direction filter in every iteration (c = 0) with a larger discard fraction, on 4 shards with the dense
    entry on every stage: ids match the oracle."""
    say(f"S=4 dense every stage, discard {discard}, cooldown 0, T {T}")
    X = mix(4000, 96, 8, 0.25, 33)
    Q = mix(400, 96, 8, 0.25, 34)
    ox = oracle.build_index(X, deg=32, S=4, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    opts = miann.SearchOptions(entry="ghost_dense", dgs=True, search_width=2, ghost_every_stage=True, t_seeds=8,
                               discard=discard, cooldown=0.0)
    g, o = run_both(ox, gx, Q, K, 32, T, opts)
    compare(g, o, label=f"S4-dense-every-stage-c0-{discard}", ndist_check=False)


def test_batches_on_two_streams():
    """Independent batches alternating over two streams, back to back (the benchmark's timing form: one batch's
    dense entry beside another's stages on 4 resident shards): every batch's ids and distance bits equal the
    single-stream search, whose ids match the oracle; so do the stage kernel's 4- and 6-wave builds."""
    say("two streams, S=4, dense entry on every stage")
    X = mix(4000, 96, 8, 0.25, 33)
    Q = mix(400, 96, 8, 0.25, 34)
    ox = oracle.build_index(X, deg=32, S=4, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    opts = miann.SearchOptions(entry="ghost_dense", dgs=True, search_width=2, ghost_every_stage=True, t_seeds=8)
    g, o = run_both(ox, gx, Q, K, 32, 9, opts)
    compare(g, o, label="S4-dense-every-stage", ndist_check=False)
    qd = dev(Q)
    ref_i, ref_d = gx.search(qd, K, 32, 9, opts)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = []
    for i in range(8):
        with torch.cuda.stream(streams[i % 2]):
            outs.append(gx.search(qd, K, 32, 9, opts))
    torch.cuda.synchronize()
    for i, (gi, gd) in enumerate(outs):
        assert torch.equal(gi, ref_i), i
        assert torch.equal(gd.view(torch.int32), ref_d.view(torch.int32)), i
    for w in (4, 6):
        ow = dataclasses.replace(opts, stage_waves=w)
        outs = []
        for i in range(4):
            with torch.cuda.stream(streams[i % 2]):
                outs.append(gx.search(qd, K, 32, 9, ow))
        torch.cuda.synchronize()
        for i, (gi, gd) in enumerate(outs):
            assert torch.equal(gi, ref_i), (w, i)
            assert torch.equal(gd.view(torch.int32), ref_d.view(torch.int32)), (w, i)


@pytest.mark.parametrize("store", ["f16", "fp8"])
def test_low_precision_parity(store):
    say(f"low precision store={store}")
    X = mix(2500, 256, 8, 0.2, 41)
    Q = mix(150, 256, 8, 0.2, 42)
    ox = oracle.build_index(X, deg=32, dgs=True, store=store, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    for kw, itopk in ((dict(), 64), (dict(dgs=True, entry="ghost_graph"), 64), (dict(entry="ghost_dense"), 40),
                      (dict(rerank_mult=8), 64)):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, itopk, 60, opts)
        compare(g, o, label=f"{store}-{kw}", ndist_check=not ghost_entry(opts))
    # traversal codes: the device quantiser matches the oracle's bit for bit
    from gpu_util import d2h
    v = gx.shard(0)
    dt = np.uint16 if store == "f16" else np.uint8
    codes = d2h(v.store, v.n * v.d_pad, dt).reshape(v.n, v.d_pad)[:, :256]
    scale = d2h(v.scale, v.n, np.float32)
    assert np.array_equal(codes, ox.shards[0]["codes"])
    assert np.array_equal(scale, ox.shards[0]["scale"])


@pytest.mark.parametrize("S", [1, 2])
def test_u8_parity_bit_exact(S):
    say(f"u8 data S={S}")
    Xf = mix(3000, 128, 8, 0.3, 51)
    X = synth.to_u8(Xf)
    Q = synth.to_u8(mix(200, 128, 8, 0.3, 52))
    ox = oracle.build_index(X, deg=32, S=S, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    for kw in (dict(), dict(dgs=True), dict(entry="ghost_graph", dgs=True), dict(entry="ghost_dense")):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, 64, 60, opts)
        frac = compare(g, o, min_frac=1.0, label=f"u8-{kw}", ndist_check=not ghost_entry(opts))
        assert frac == 1.0


def test_sign_table_parity(small):
    from gpu_util import d2h
    X, Q, ox, gx = small
    v = gx.shard(0)
    S = d2h(v.sign, v.n * v.W * v.degree, np.uint32).reshape(v.n, v.W, v.degree)
    assert np.array_equal(S.transpose(0, 2, 1), ox.shards[0]["sign"])


def test_batch_independence_and_query_keys(small):
    """A query's result depends on its key, not on its batch (serving requirement)."""
    X, Q, ox, gx = small
    opts = miann.SearchOptions(dgs=True, entry="ghost_graph")
    full = gx.search(dev(Q), K, 64, 60, opts)
    sub = np.arange(7, 300, 5)
    part = gx.search(dev(Q[sub]), K, 64, 60, opts, qkeys=torch.from_numpy(sub.astype(np.int64)).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(full[0].cpu().numpy()[sub], part[0].cpu().numpy())
    assert np.array_equal(full[1].cpu().numpy()[sub], part[1].cpu().numpy())


def test_phase_events_pipelined(small):
    """Caller events recorded in stream order around the entry, the stages and the merge: three
    back-to-back calls without a wait return the results of a plain call, and the intervals are
    ordered and non-negative."""
    import ctypes
    X, Q, ox, gx = small
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    evs = []
    for _ in range(12):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    opts = miann.SearchOptions(dgs=True, entry="ghost_dense", search_width=2)
    qd = dev(Q)
    ref = gx.search(qd, K, 64, 40, opts)
    outs = [gx.search(qd, K, 64, 40, opts, phase_events=evs[4 * i:4 * i + 4]) for i in range(3)]
    torch.cuda.synchronize()
    for ids, dists in outs:
        assert torch.equal(ids, ref[0]) and torch.equal(dists, ref[1])
    ms = ctypes.c_float()
    for i in range(3):
        for j in range(3):
            assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[4 * i + j], evs[4 * i + j + 1]) == 0
            assert ms.value >= 0.0
        assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[4 * i], evs[4 * i + 3]) == 0 and ms.value > 0.0
    for e in evs:
        hip.hipEventDestroy(e)


def test_concurrent_calls_on_one_stream(small):
    """Host threads searching on the same stream at once: a call that finds the stream's kept scratch
    held by another thread takes its own block, so every call returns the single-call result."""
    import threading
    X, Q, ox, gx = small
    opts = miann.SearchOptions(dgs=True, entry="ghost_dense", search_width=2)
    qd = dev(Q)
    ref = gx.search(qd, K, 64, 40, opts)
    torch.cuda.synchronize()
    out = [None] * 4

    def work(i):
        out[i] = [gx.search(qd, K, 64, 40, opts) for _ in range(3)]

    th = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    for calls in out:
        for ids, dists in calls:
            assert torch.equal(ids, ref[0]) and torch.equal(dists, ref[1])


def test_per_query_budget_and_seed_entry(small):
    X, Q, ox, gx = small
    rng = np.random.default_rng(3)
    Tq = rng.integers(0, 90, len(Q)).astype(np.int32)
    seeds = rng.integers(0, len(X), (len(Q), 24)).astype(np.uint32)
    opts = miann.SearchOptions(entry="seeds", dgs=True)
    g, o = run_both(ox, gx, Q, K, 64, 80, opts, seeds=seeds, Tq=Tq)
    compare(g, o, label="seeds+Tq")


def test_full_tiny_workload():
    """The tiny configuration at full size: N = 10,000, d = 128, 32 components, degree 32,
    1,000 queries, k = 10, itopk = 64."""
    say("tiny workload N=10000 nq=1000")
    X = synth.mixture_small(10_000, 128, 32, 0.3, synth.SEED_BASE)
    Q = synth.mixture_small(1000, 128, 32, 0.3, synth.SEED_QUERIES)
    ox = oracle.build_index(X, deg=32, dgs=True, ghost_ratio=0.01, deg_g=32)
    gx = to_device_index(ox)
    for kw in (dict(), dict(n_init=256), dict(entry="ghost_dense", dgs=True), dict(entry="ghost_graph", dgs=True)):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox, gx, Q, K, 64, 64, opts)
        compare(g, o, label=f"tiny-{kw}", ndist_check=not ghost_entry(opts))


def test_validation_errors(small):
    X, Q, ox, gx = small
    q = dev(Q[:4])
    with pytest.raises(miann.MiannError) as e:
        gx.search(q, 20, 10, 10)
    assert e.value.status == 1
    with pytest.raises(miann.MiannError):
        gx.search(q, 10, 600, 10)
    with pytest.raises(miann.MiannError):
        gx.search(q, 10, 64, 10, miann.SearchOptions(search_width=3))  # 3 * 32 > 64
    with pytest.raises(miann.MiannError):
        gx.search(q, 10, 64, 10, miann.SearchOptions(hash_log2=7))
    for w in (3, 7):
        with pytest.raises(miann.MiannError) as e:
            gx.search(q, 10, 64, 10, miann.SearchOptions(stage_waves=w))
        assert "stage_waves" in str(e.value)
    ids, dists = gx.search(dev(Q[:0]), 10, 64, 10)
    assert ids.shape == (0, 10)
