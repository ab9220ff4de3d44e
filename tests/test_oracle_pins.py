"""Pins for the CPU oracle: each test ties an oracle function to something other
than itself (a textbook routine, a closed form, an invariant the paper's
algorithm implies, a published test vector, or brute force on a tiny input).

Paper references: Sec. 2.1 Eq. 1 (k-NN), Sec. 2.2 Eq. 2 and Steps 1-4 (beam
search), Sec. 3.1.2 (I(u) and the staged search), Sec. 3.2.2 (ghost staging),
Sec. 3.3.2 / Sec. 4 (direction table and selection), Sec. 5.1 (Recall@k).
"""
import math
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import breadth_first_order, connected_components

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def f32_order(D64, k):
    """Brute force order by (f32(dist), id) from float64 squared distances (numpy)."""
    D32 = np.asarray(D64).astype(np.float32)
    n = D32.shape[1]
    return np.stack([np.lexsort((np.arange(n), row))[:k] for row in D32])


def small(n=400, d=16, C=4, sigma=0.3, seed=1):
    return synth.mixture_small(n, d, C, sigma, seed)


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------
def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if not x.startswith("#")]
    seed, expect = vals[0], vals[1:]
    assert [oracle.splitmix(seed, i + 1) for i in range(5)] == expect


def test_keyed_order_is_permutation_and_partition_covers():
    perm = oracle.keyed_order(123, 1000)
    assert sorted(perm.tolist()) == list(range(1000))
    assert not np.array_equal(perm, np.arange(1000))
    parts = oracle.partition(1001, 4, 5)
    allids = np.concatenate(parts)
    assert sorted(allids.tolist()) == list(range(1001))
    assert [len(p) for p in parts] == [(s + 1) * 1001 // 4 - s * 1001 // 4 for s in range(4)]
    assert np.array_equal(oracle.partition(50, 1, 5)[0], np.arange(50))


def test_ghost_sample_uniform_without_replacement():
    g = oracle.ghost_sample(10000, 500, 9, 0)
    assert len(np.unique(g)) == 500 and np.all(np.diff(g.astype(np.int64)) > 0) and g.max() < 10000
    # roughly uniform: counts per decile within 5 sigma of 50
    h = np.histogram(g, bins=10, range=(0, 10000))[0]
    assert np.all(np.abs(h - 50) < 5 * np.sqrt(50))


# ---------------------------------------------------------------------------
# Eq. 2 (squared) and Eq. 1
# ---------------------------------------------------------------------------
def test_distance_matches_float_differences_summed_in_double():
    X = small(50, 37)
    q = small(1, 37, seed=2)[0]
    for v in range(50):
        diff = (q - X[v]).astype(np.float32)  # numpy float32 subtraction, rounded to nearest
        ref = np.float32(math.fsum((diff.astype(np.float64) ** 2).tolist()))
        assert oracle.dist(X, q, v) == float(ref)


def test_distance_u8_exact():
    rng = np.random.default_rng(0)
    X = rng.integers(0, 256, (20, 128)).astype(np.uint8)
    q = rng.integers(0, 256, 128).astype(np.uint8)
    for v in range(20):
        assert oracle.dist(X, q, v) == float(((q.astype(np.int64) - X[v].astype(np.int64)) ** 2).sum())
    # the largest possible value fits int32
    X0 = np.zeros((1, 128), np.uint8)
    q255 = np.full(128, 255, np.uint8)
    assert oracle.dist(X0, q255, 0) == 255 * 255 * 128


@pytest.mark.parametrize("k", [1, 7, 30])
def test_exact_knn_equals_numpy_brute_force(k):
    X = small(300, 24)
    Q = small(40, 24, seed=2)
    ids, ds = oracle.knn(X, Q, k)
    _, D = oracle.brute_force_numpy(X, Q, k)
    assert np.array_equal(ids, f32_order(D, k))
    assert np.array_equal(ds.astype(np.float32), np.take_along_axis(D, ids.astype(np.int64), 1).astype(np.float32))


def test_exact_knn_u8_ties_broken_by_id():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 4, (200, 8)).astype(np.uint8)  # many exact ties
    Q = rng.integers(0, 4, (10, 8)).astype(np.uint8)
    ids, ds = oracle.knn(X, Q, 20)
    D = ((Q[:, None, :].astype(np.int64) - X[None].astype(np.int64)) ** 2).sum(-1)
    for i in range(10):
        assert ids[i].tolist() == np.lexsort((np.arange(200), D[i]))[:20].tolist()


def test_knn_exclude_self():
    X = small(100, 8)
    ids, _ = oracle.knn(X, X, 5, exclude_self=True)
    assert not np.any(ids == np.arange(100)[:, None])


def test_recall_closed_form():
    gt = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    ann = np.array([[4, 3, 9, 9], [5, 6, 7, 8]])
    assert oracle.recall(gt, ann, 4) == (2 + 4) / 8


# ---------------------------------------------------------------------------
# Graph: k-NN lists pruned to a fixed degree (reverse-merge rule)
# ---------------------------------------------------------------------------
def test_prune_rule_properties():
    X = small(300, 12)
    deg, K0 = 8, 16
    knn_ids, knn_d = oracle.knn(X, X, K0, exclude_self=True)
    G = oracle.prune(X, knn_ids, knn_d, deg)
    half = (deg + 1) // 2
    rev = [set() for _ in range(300)]
    for v in range(300):
        for u in knn_ids[v, :half]:
            rev[u].add(v)
    for u in range(300):
        row = G[u].tolist()
        assert len(set(row)) == deg and u not in row
        dd = [oracle.dist(X, X[u], v) for v in row]
        assert all((dd[i], row[i]) < (dd[i + 1], row[i + 1]) for i in range(deg - 1))
        F = set(knn_ids[u, :half].tolist())
        assert F <= set(row)
        # reverse candidates (nearest first) come before the k-NN tail
        rc = sorted(rev[u] - F, key=lambda v: (oracle.dist(X, X[u], v), v))
        expect = list(F) + rc[: deg - half]
        tail = [v for v in knn_ids[u, half:].tolist() if v not in set(expect)]
        expect = expect + tail[: deg - len(expect)]
        assert set(row) == set(expect)


# ---------------------------------------------------------------------------
# Direction table (Sec. 3.3.2 (a)) and query sign bits
# ---------------------------------------------------------------------------
def test_sign_table_unit_vectors():
    d = 70  # W = 3, with pad bits
    X = np.zeros((d + 1, d), np.float32)
    for i in range(d):
        X[i + 1, i] = 1.0
    G = np.array([[i + 1 for i in range(d)]] + [[0] * d for _ in range(d)], np.uint32)
    S = oracle.sign_table(X, G)
    W = (d + 31) // 32
    assert S.shape == (d + 1, d, W)
    for j in range(d):  # edge 0 -> e_j: exactly bit j set
        expect = np.zeros(W, np.uint32)
        expect[j // 32] = np.uint32(1 << (j % 32))
        assert np.array_equal(S[0, j], expect)
    for u in range(1, d + 1):  # edge e_i -> 0: no coordinate grows
        assert not S[u].any()


def test_sign_table_reverse_edge_complement_and_popcount():
    X = small(200, 40)
    G = oracle.build_graph(X, 8)
    S = oracle.sign_table(X, G)
    W = 2
    valid = np.array([0xFFFFFFFF, (1 << 8) - 1], np.uint32)
    pairs = 0
    for u in range(200):
        for j, v in enumerate(G[u]):
            cnt = sum(bin(int(w)).count("1") for w in S[u, j])
            assert cnt == int((X[v] > X[u]).sum())
            assert (S[u, j] & ~valid).sum() == 0  # pad bits stay zero
            back = np.where(G[v] == u)[0]
            if len(back):
                pairs += 1
                neq = X[v] != X[u]
                x = S[u, j] ^ S[v, back[0]]
                assert sum(bin(int(w)).count("1") for w in x) == int(neq.sum())
    assert pairs > 0


# ---------------------------------------------------------------------------
# Beam search
# ---------------------------------------------------------------------------
def reachable_from(G, starts):
    n = G.shape[0]
    A = csr_matrix((np.ones(G.size), (np.repeat(np.arange(n), G.shape[1]), G.ravel().astype(np.int64))), shape=(n, n))
    seen = set()
    for s in starts:
        if s not in seen:
            seen |= set(breadth_first_order(A, int(s), directed=True, return_predecessors=False).tolist())
    return np.array(sorted(seen))


def init_ids(seed, shard, qkey, n_init, n):
    st = int(oracle.lib().orc_stream_main(seed, shard))
    return [oracle.splitmix(st, qkey * n_init + j + 1) % n for j in range(n_init)]


def test_pin1_exhaustive_search_is_brute_force_over_reachable():
    X = small(300, 16, C=3)
    Q = small(25, 16, C=3, seed=2)
    ix = oracle.build_index(X, deg=8, dgs=False)
    G = ix.shards[0]["graph"]
    ids, ds, ctr = oracle.search(ix, Q, k=10, l=300, T=400, n_init=4)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    for i in range(25):
        reach = reachable_from(G, init_ids(6, 0, i, 4, 300))
        sub = D[i, reach].astype(np.float32)
        order = reach[np.lexsort((reach, sub))][:10]
        assert ids[i, : len(order)].tolist() == order.tolist()
        assert np.all(ds[i] == np.sort(ds[i]))


def test_pin1_connected_graph_full_brute_force():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((250, 10)).astype(np.float32)  # one blob: connected k-NN graph
    Q = rng.standard_normal((20, 10)).astype(np.float32)
    ix = oracle.build_index(X, deg=10, dgs=False)
    G = ix.shards[0]["graph"]
    n_cc = connected_components(csr_matrix((np.ones(G.size), (np.repeat(np.arange(250), 10), G.ravel().astype(np.int64))),
                                           shape=(250, 250)), directed=True, connection="strong")[0]
    assert n_cc == 1
    ids, ds, _ = oracle.search(ix, Q, k=10, l=250, T=300)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    assert np.array_equal(ids, f32_order(D, 10))


def test_pin2_outputs_sorted_and_distances_recomputed():
    X = small(500, 20)
    Q = small(30, 20, seed=2)
    ix = oracle.build_index(X, deg=8, dgs=True, ghost_ratio=0.05, deg_g=8)
    for kw in [dict(), dict(dgs_on=True), dict(entry="ghost_graph"), dict(entry="ghost_dense", dgs_on=True, r=2)]:
        ids, ds, _ = oracle.search(ix, Q, k=10, l=32, T=40, **kw)
        for i in range(30):
            keys = [(float(ds[i, j]), int(ids[i, j])) for j in range(10)]
            assert keys == sorted(keys)
            for j in range(10):
                ref = np.float32((((Q[i] - X[ids[i, j]]).astype(np.float32).astype(np.float64)) ** 2).sum())
                assert ds[i, j] == ref


@pytest.mark.parametrize("kw", [dict(), dict(dgs_on=True), dict(r=2), dict(dgs_on=True, r=3, entry="ghost_graph")])
def test_pin4_visited_policy_does_not_change_results(kw):
    X = small(800, 16, C=6)
    Q = small(40, 16, C=6, seed=2)
    ix = oracle.build_index(X, deg=12, dgs=True, ghost_ratio=0.05, deg_g=8)
    base = oracle.search(ix, Q, k=10, l=24, T=60, **kw)
    for pol in ("forget_each_iter", "small_hash"):
        other = oracle.search(ix, Q, k=10, l=24, T=60, visited=pol, **kw)
        assert np.array_equal(base[0], other[0]) and np.array_equal(base[1], other[1])
        # expansions and iterations are identical; only the distance count may grow
        assert np.array_equal(base[2][:, 1:4], other[2][:, 1:4])
        assert np.all(other[2][:, 0] >= base[2][:, 0])
        assert other[2][:, 0].sum() > base[2][:, 0].sum()


def test_pin5_special_cases_reduce_to_plain():
    X = small(600, 16, C=5)
    Q = small(30, 16, C=5, seed=2)
    ix = oracle.build_index(X, deg=10, dgs=True)
    plain = oracle.search(ix, Q, k=10, l=32, T=50)
    for kw in [dict(dgs_on=True, discard=0.0), dict(dgs_on=True, cooldown=1.0), dict(ppe_on=False)]:
        o = oracle.search(ix, Q, k=10, l=32, T=50, **kw)
        assert np.array_equal(plain[0], o[0]) and np.array_equal(plain[1], o[1])
        assert np.array_equal(plain[2][:, :3], o[2][:, :3])
    # DGS on with discard > 0 really changes the work done
    o = oracle.search(ix, Q, k=10, l=32, T=50, dgs_on=True)
    assert o[2][:, 3].sum() > 0


def test_ghost_every_stage_reduces_to_stage0_entry_without_path_extension():
    X = small(600, 16, C=5)
    Q = small(30, 16, C=5, seed=2)
    ix1 = oracle.build_index(X, deg=10, dgs=True, ghost_ratio=0.1, deg_g=8)
    for e in ("ghost_graph", "ghost_dense"):
        a = oracle.search(ix1, Q, k=5, l=32, T=30, entry=e)
        b = oracle.search(ix1, Q, k=5, l=32, T=30, entry=e, ghost_every_stage=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    ix3 = oracle.build_index(X, deg=10, S=3, dgs=True, ghost_ratio=0.1, deg_g=8)
    a = oracle.search(ix3, Q, k=5, l=32, T=30, entry="ghost_dense", ppe_on=False)
    b = oracle.search(ix3, Q, k=5, l=32, T=30, entry="ghost_dense", ppe_on=False, ghost_every_stage=True)
    assert np.array_equal(a[0], b[0])
    # with path extension, later stages do extra ghost work
    a = oracle.search(ix3, Q, k=5, l=32, T=30, entry="ghost_dense")
    b = oracle.search(ix3, Q, k=5, l=32, T=30, entry="ghost_dense", ghost_every_stage=True)
    assert np.all(b[2][:, 4] == 3 * a[2][:, 4])


def test_pin5_dense_ghost_over_all_nodes_is_brute_force():
    X = small(200, 12, C=4)
    Q = small(20, 12, C=4, seed=2)
    ix = oracle.build_index(X, deg=8, dgs=False, ghost_R=200, deg_g=8)
    assert np.array_equal(ix.shards[0]["g_map"], np.arange(200))
    ids, ds, ctr = oracle.search(ix, Q, k=10, l=40, T=0, entry="ghost_dense", t_seeds=40)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    assert np.array_equal(ids, f32_order(D, 10))
    assert np.all(ctr[:, 4] == 200)


def test_pin13_dgs_worked_example_shape():
    """Sec. 3.3.2 example: visiting node 5 with n = 2 keeps the two neighbours that
    point toward the query (9 and 6); sorting gives 9, 6, 5; r = 1 next picks 9."""
    X = np.zeros((12, 2), np.float32)
    X[5] = [0.0, 0.0]
    X[9] = [2.0, 2.0]   # toward the query, nearest to it
    X[6] = [1.0, 1.5]   # toward the query
    X[2] = [-1.0, -1.0] # away
    X[3] = [-0.5, 1.0]  # mixed
    for i, v in enumerate([0, 1, 4, 7, 8, 10, 11]):
        X[v] = [-5.0 - i, -5.0]
    q = np.array([[3.0, 3.0]], np.float32)
    G = np.zeros((12, 4), np.uint32)
    G[5] = [2, 3, 6, 9]
    for u in range(12):
        if u != 5:
            G[u] = [5, 2, 3, 6] if u != 5 else G[u]
    G[9] = [5, 6, 2, 3]
    ix = oracle.build_index(X, deg=4, dgs=True, graph=G)
    S = ix.shards[0]["sign"]
    assert S[5, 3, 0] == 0b11 and S[5, 2, 0] == 0b11 and S[5, 0, 0] == 0
    ids, ds, ctr = oracle.search(ix, q, k=3, l=3, T=1, entry="seeds", seeds=np.array([[5]]),
                                 dgs_on=True, discard=0.5, cooldown=0.0, n_init=1)
    assert ids[0].tolist() == [9, 6, 5]
    assert ctr[0, 0] == 3 and ctr[0, 3] == 2 and ctr[0, 1] == 1
    # second iteration expands node 9 (the first fresh entry); its DGS picks are
    # already visited or pointing away, so nothing new enters.
    ids2, _, ctr2 = oracle.search(ix, q, k=3, l=3, T=2, entry="seeds", seeds=np.array([[5]]),
                                  dgs_on=True, discard=0.5, cooldown=0.0, n_init=1)
    assert ids2[0].tolist() == [9, 6, 5] and ctr2[0, 1] == 2


def test_dgs_cooldown_and_forced_cooldown_counts():
    X = small(400, 16, C=3)
    Q = small(10, 16, C=3, seed=2)
    ix = oracle.build_index(X, deg=8, dgs=True)
    T = 40
    _, _, c = oracle.search(ix, Q, k=5, l=16, T=T, dgs_on=True, discard=0.5, cooldown=0.3)
    n_dgs_iters = T - int(np.ceil(0.3 * T))
    # every DGS-phase expansion skips exactly floor(0.5 * 8) = 4 slots
    assert np.all(c[:, 3] % 4 == 0) and np.all(c[:, 3] <= 4 * n_dgs_iters)


def test_random_discard_ablation_differs_from_dgs():
    X = small(800, 32, C=5)
    Q = small(40, 32, C=5, seed=2)
    ix = oracle.build_index(X, deg=12, dgs=True)
    a = oracle.search(ix, Q, k=10, l=32, T=60, dgs_on=True)
    b = oracle.search(ix, Q, k=10, l=32, T=60, dgs_on=True, random_discard=True)
    assert not np.array_equal(a[0], b[0])
    assert np.array_equal(a[2][:, 3] > 0, b[2][:, 3] > 0)


# ---------------------------------------------------------------------------
# Path extension over shards (Sec. 3.1.2)
# ---------------------------------------------------------------------------
def test_pin7_inter_shard_map_is_brute_force_1nn():
    X = small(400, 12, C=3)
    ix = oracle.build_index(X, deg=8, S=3, dgs=False)
    for s in range(3):
        A = ix.shards[s]["orig_base"]
        B = ix.shards[(s + 1) % 3]["orig_base"]
        _, D = oracle.brute_force_numpy(B, A, 1)
        assert np.array_equal(ix.shards[s]["next"], f32_order(D, 1)[:, 0])


def test_ppe_exhaustive_stages_merge_to_global_brute_force():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((360, 8)).astype(np.float32)
    Q = rng.standard_normal((15, 8)).astype(np.float32)
    ix = oracle.build_index(X, deg=10, S=3, dgs=False)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    for ppe in (True, False):
        ids, ds, ctr = oracle.search(ix, Q, k=10, l=120, T=200, ppe_on=ppe)
        assert np.array_equal(ids, f32_order(D, 10))


def test_ppe_handoff_chain_with_zero_iterations():
    """With T = 0 each stage only evaluates its seeds: stage 0 the random start
    nodes, stage t the single node I(z) handed over (f = 1). The merged result is
    the chain z0, I(z0), I(I(z0)) ... in global ids, sorted."""
    X = small(300, 8, C=3)
    Q = small(6, 8, C=3, seed=2)
    S = 3
    ix = oracle.build_index(X, deg=8, S=S, dgs=False)
    ids, ds, ctr = oracle.search(ix, Q, k=3, l=8, T=0, n_init=1)
    for i in range(6):
        s0 = i % S
        sh = ix.shards[s0]
        starts = init_ids(6, s0, i, 1, sh["n"])
        dd = [(oracle.dist(sh["orig_base"], Q[i], v), v) for v in set(starts)]
        z = min(dd)[1]
        chain = [(float(np.float32(min(dd)[0])), int(sh["gmap"][z]))]
        s = s0
        for _ in range(S - 1):
            z = int(ix.shards[s]["next"][z])
            s = (s + 1) % S
            chain.append((float(np.float32(oracle.dist(ix.shards[s]["orig_base"], Q[i], z))), int(ix.shards[s]["gmap"][z])))
        chain.sort()
        assert ids[i].tolist() == [c[1] for c in chain]
        assert ctr[i, 2] == 0


# ---------------------------------------------------------------------------
# Number formats and low-precision traversal
# ---------------------------------------------------------------------------
def test_pin8_fp8_decode_all_codes_vs_torch():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.fp8_decode(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    same = (ours == ref) | (np.isnan(ours) & np.isnan(ref))
    assert same.all()
    assert np.nanmax(ours) == 448.0 and np.isnan(ours[0x7F]) and np.isnan(ours[0xFF])


def test_pin8_f16_decode_all_codes_vs_numpy():
    codes = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ours = oracle.f16_decode(codes)
    ref = codes.view(np.float16).astype(np.float32)
    assert ((ours == ref) | (np.isnan(ours) & np.isnan(ref))).all()


def test_pin8_encoders_round_to_nearest_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(3000) * 50, rng.standard_normal(2000) * 1e-2,
                        rng.uniform(-447, 447, 1000)]).astype(np.float32)
    ours = oracle.fp8_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    # exact midpoints between consecutive codes go to the even code
    vals = oracle.fp8_decode(np.arange(127, dtype=np.uint8)).astype(np.float64)
    mids = ((vals[:-1] + vals[1:]) / 2).astype(np.float32)
    enc = oracle.fp8_encode(mids)
    assert np.all(enc % 2 == 0)
    assert oracle.fp8_encode(np.array([1e6, -1e6], np.float32)).tolist() == [126, 254]  # saturate
    h = oracle.f16_encode(x)
    assert np.array_equal(h, x.astype(np.float16).view(np.uint16))


def test_quantize_scale_and_error_bound():
    X = small(50, 64)
    X[3] = 0
    codes, scale = oracle.quantize(X, "fp8")
    assert scale[3] == 1.0 and not codes[3].any()
    xt = oracle.dequantize(codes, scale, "fp8")
    mx = np.abs(X).max(1)
    # the largest element maps to +-448 exactly
    for v in range(50):
        if v != 3:
            assert np.abs(oracle.fp8_decode(codes[v])).max() == 448.0
    # e4m3 relative rounding error <= 2^-4 in the normal range, absolute 2^-10 * s below it
    err = np.abs(xt - X)
    bound = np.maximum(np.abs(X) * 2.0 ** -4, (scale[:, None] * 2.0 ** -10)) * 1.0001 + 1e-12
    assert np.all(err <= bound)
    c16, s16 = oracle.quantize(X, "f16")
    assert np.all(s16 == 1.0) and np.array_equal(c16, X.astype(np.float16).view(np.uint16))


def test_low_precision_rerank_exhaustive_matches_f32_brute_force():
    X = small(300, 32, C=3)
    Q = small(20, 32, C=3, seed=2)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    exact = f32_order(D, 10)
    for store in ("f16", "fp8"):
        ix = oracle.build_index(X, deg=10, dgs=False, store=store)
        assert ix.shards[0]["codes"].dtype == (np.uint16 if store == "f16" else np.uint8)
        ids, ds, ctr = oracle.search(ix, Q, k=10, l=300, T=400, n_init=300)
        # traversal top-40 under the low-precision distance, reranked in f32
        xt = oracle.dequantize(ix.shards[0]["codes"], ix.shards[0]["scale"], store)
        _, Dl = oracle.brute_force_numpy(xt, Q, 40)
        for i in range(20):
            top40 = f32_order(Dl[i:i + 1], 40)[0]
            sub = D[i, top40].astype(np.float32)
            expect = top40[np.lexsort((top40, sub))][:10]
            assert ids[i].tolist() == expect.tolist()
            assert np.all(ds[i] == D[i, ids[i]].astype(np.float32))
        assert np.all(ctr[:, 6] == 40)
        assert oracle.recall(exact, ids, 10) >= 0.9


def test_u8_search_exact_int_distances():
    rng = np.random.default_rng(4)
    Xf = synth.mixture_small(400, 32, 3, 0.3, 1)
    X = synth.to_u8(Xf)
    Q = synth.to_u8(synth.mixture_small(10, 32, 3, 0.3, 2))
    ix = oracle.build_index(X, deg=8, dgs=True)
    ids, ds, _ = oracle.search(ix, Q, k=5, l=32, T=40, dgs_on=True)
    assert ds.dtype == np.int32
    for i in range(10):
        for j in range(5):
            assert ds[i, j] == int(((Q[i].astype(np.int64) - X[ids[i, j]].astype(np.int64)) ** 2).sum())


def test_degenerate_inputs():
    X = small(60, 8)
    ix = oracle.build_index(X, deg=4, dgs=True)
    ids, ds, ctr = oracle.search(ix, np.zeros((0, 8), np.float32), k=3, l=8, T=5)
    assert ids.shape == (0, 3)
    # k == l, T == 0 (initial candidates only)
    ids, ds, ctr = oracle.search(ix, X[:3], k=8, l=8, T=0)
    assert np.all(ctr[:, 2] == 0) and np.all(ds[:, 0] >= 0)
    with pytest.raises(ValueError):
        oracle.search(ix, X[:3], k=9, l=8, T=5)


# ---------------------------------------------------------------------------
# Eq. 2 against its exact value. The oracle's distance is the float32
# difference of each coordinate, squared and summed in double, rounded once to
# float. Relative to the exact sum of (q_i - x_i)^2 that differs by at most
#   2^-23 + 2^-48   (each difference rounded to float, then squared)
# + d * 2^-53       (the double sum of non-negative terms)
# + 2^-24           (the final rounding to float),
# which the bound below rounds up to 3 * 2^-24 + d * 2^-52.
# ---------------------------------------------------------------------------
def _exact_sq_l2(q, x):
    from fractions import Fraction
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(q, x))


@pytest.mark.parametrize("d,scale", [(7, 1.0), (96, 0.25), (128, 30.0), (256, 1e-3), (300, 1e4)])
def test_distance_within_rounding_bound_of_exact_eq2(d, scale):
    rng = np.random.default_rng(d)
    X = (rng.standard_normal((40, d)) * scale).astype(np.float32)
    q = (rng.standard_normal(d) * scale).astype(np.float32)
    X[0] = q                      # distance 0 exactly
    X[1] = q + np.float32(scale)  # every coordinate differs by about the same amount
    bound = 3 * 2.0 ** -24 + d * 2.0 ** -52
    for v in range(40):
        exact = _exact_sq_l2(q, X[v])
        got = oracle.dist(X, q, v)
        if exact == 0:
            assert got == 0.0
            continue
        rel = abs(float((got - exact) / exact))
        assert rel <= bound, (v, rel, bound)


def test_distance_correctly_rounded_when_differences_are_exact():
    """Coordinates on a grid of 2^-6 in [-8, 8]: every float difference and its
    square are exact, so the oracle must return the exact sum rounded once to the
    nearest float."""
    rng = np.random.default_rng(17)
    d = 129
    X = (rng.integers(-512, 513, (60, d)) / 64.0).astype(np.float32)
    q = (rng.integers(-512, 513, d) / 64.0).astype(np.float32)
    for v in range(60):
        exact = _exact_sq_l2(q, X[v])
        assert exact.denominator <= 1 << 12
        assert oracle.dist(X, q, v) == float(np.float32(float(exact)))


# ---------------------------------------------------------------------------
# Direction-guided selection and its cool-down (Sec. 3.3.2 (b)): entries that a
# DGS expansion only partly expanded are expanded again, in full, once the
# cool-down starts; the cool-down is the last ceil(c T) iterations, and starts
# early when no fresh entry is left.
# ---------------------------------------------------------------------------
def _kept_edge_reach(X, G, S, q, starts, n_keep):
    """Nodes reachable from `starts` when every node follows only its n_keep slots of
    smallest (sign mismatch, slot) toward query q (numpy, independent of oracle.c)."""
    d = X.shape[1]
    seen = set(int(s) for s in starts)
    todo = list(seen)
    while todo:
        u = todo.pop()
        qbits = (q > X[u])
        mm = []
        for j in range(G.shape[1]):
            vbits = np.array([(int(S[u, j, i // 32]) >> (i % 32)) & 1 for i in range(d)], bool)
            mm.append((int((qbits != vbits).sum()), j))
        for _, j in sorted(mm)[:n_keep]:
            v = int(G[u, j])
            if v not in seen:
                seen.add(v)
                todo.append(v)
    return seen


def test_dgs_exhaustive_search_reaches_brute_force_through_the_cooldown():
    """l >= N and a budget large enough for every node to be expanded in full after
    the direction-filtered phase: on a connected graph the result is brute force.
    The nodes reachable through the kept slots alone miss part of the true top-10
    for some queries, so a cool-down that did not re-expand partly expanded entries
    could not reach it."""
    rng = np.random.default_rng(8)
    N, d = 160, 12
    X = rng.standard_normal((N, d)).astype(np.float32)
    Q = rng.standard_normal((25, d)).astype(np.float32)
    ix = oracle.build_index(X, deg=8, dgs=True)
    G, S = ix.shards[0]["graph"], ix.shards[0]["sign"]
    n_cc = connected_components(csr_matrix((np.ones(G.size), (np.repeat(np.arange(N), 8), G.ravel().astype(np.int64))),
                                           shape=(N, N)), directed=True, connection="strong")[0]
    assert n_cc == 1
    T = 4 * N
    ids, ds, ctr = oracle.search(ix, Q, k=10, l=N, T=T, n_init=2, dgs_on=True, discard=0.5, cooldown=0.3)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    truth = f32_order(D, 10)
    assert np.array_equal(ids, truth)
    assert np.all(ctr[:, 3] > 0)
    short = 0
    for i in range(len(Q)):
        reach = _kept_edge_reach(X, G, S, Q[i], init_ids(6, 0, i, 2, N), 4)
        short += not set(truth[i].tolist()) <= reach
    assert short > 0


def _line_index(pos, G):
    X = np.asarray(pos, np.float32).reshape(-1, 1)
    return X, oracle.build_index(X, deg=G.shape[1], dgs=True, graph=np.asarray(G, np.uint32))


def test_dgs_cooldown_length_is_ceil_of_c_times_T():
    """A chain 0 - 1 - ... - 11 on a line, query far to the right, seed 0. Each DGS
    expansion keeps the one slot that points right, so the search walks one node per
    iteration. T = 9, c = 0.3: the cool-down is ceil(2.7) = 3 iterations, so exactly 6
    expansions run under the filter (floor would give 7)."""
    n = 12
    G = [[1, 2]] + [[i - 1, i + 1] for i in range(1, n - 1)] + [[n - 2, n - 3]]
    X, ix = _line_index(range(n), np.array(G))
    q = np.array([[20.0]], np.float32)
    ids, ds, ctr = oracle.search(ix, q, k=3, l=n, T=9, entry="seeds", seeds=np.array([[0]]), dgs_on=True,
                                 discard=0.5, cooldown=0.3)
    assert ids[0].tolist() == [9, 8, 7]
    assert ctr[0, 3] == 6      # slots skipped: one per DGS-phase expansion
    assert ctr[0, 1] == 9 and ctr[0, 2] == 9 and ctr[0, 0] == 10


def test_dgs_forced_cooldown_reexpands_partial_entries():
    """Nodes on a line: A = 0, B = 1, C = 2, D = 10; query 11; seed A.
    A -> (B, D): both point toward the query, the slot order keeps B and skips D.
    B -> (A, C) keeps C. C -> (B, A) keeps B, already visited: no fresh entry is left
    after three DGS iterations, so the cool-down starts at once without spending an
    iteration. It expands C, B and A in full (they were partial); A's skipped slot
    finally reaches D, which is expanded in the last of the T = 7 iterations."""
    G = np.array([[1, 3], [0, 2], [1, 0], [2, 0]])
    X, ix = _line_index([0.0, 1.0, 2.0, 10.0], G)
    q = np.array([[11.0]], np.float32)
    ids, ds, ctr = oracle.search(ix, q, k=3, l=4, T=7, entry="seeds", seeds=np.array([[0]]), dgs_on=True,
                                 discard=0.5, cooldown=0.3)
    assert ids[0].tolist() == [3, 2, 1]
    assert ds[0].tolist() == [1.0, 81.0, 100.0]
    assert ctr[0, 0] == 4 and ctr[0, 1] == 7 and ctr[0, 2] == 7 and ctr[0, 3] == 3
    # one iteration less: D is found but not expanded
    _, _, c6 = oracle.search(ix, q, k=3, l=4, T=6, entry="seeds", seeds=np.array([[0]]), dgs_on=True,
                             discard=0.5, cooldown=0.3)
    assert c6[0, 1] == 6 and c6[0, 0] == 4


# ---------------------------------------------------------------------------
# Ghost staging hands over M[g], the node a ghost copies (Sec. 3.2.2).
# ---------------------------------------------------------------------------
def _ghost_expect(X, q, gmap, t):
    Xg = np.ascontiguousarray(X[gmap])
    _, Dg = oracle.brute_force_numpy(Xg, q[None], 1)
    top = f32_order(Dg, t)[0]
    nodes = gmap[top].astype(np.int64)
    _, D = oracle.brute_force_numpy(X, q[None], 1)
    dn = D[0, nodes].astype(np.float32)
    order = np.lexsort((nodes, dn))
    return top, nodes[order], dn[order]


@pytest.mark.parametrize("entry", ["ghost_dense", "ghost_graph"])
def test_ghost_seeds_are_the_mapped_nodes_of_the_nearest_ghosts(entry):
    """R = 60 ghosts out of N = 500, so the ghost index and the node it copies differ.
    With T = 0 the result is exactly the handed-over seeds: the nodes M[g] of the t
    ghosts nearest to the query (exact for the dense entry; for the graph entry an
    exhaustive ghost search on a connected ghost graph), ordered by (dist, id)."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((500, 10)).astype(np.float32)
    Q = rng.standard_normal((20, 10)).astype(np.float32)
    ix = oracle.build_index(X, deg=8, dgs=False, ghost_R=60, deg_g=8)
    gmap = ix.shards[0]["g_map"]
    assert len(gmap) == 60 and np.any(gmap != np.arange(60))
    t = 12
    kw = dict(l_g=60, T_g=200) if entry == "ghost_graph" else {}
    if entry == "ghost_graph":
        Gg = ix.shards[0]["g_graph"]
        assert connected_components(csr_matrix((np.ones(Gg.size), (np.repeat(np.arange(60), 8),
                                                                    Gg.ravel().astype(np.int64))), shape=(60, 60)),
                                    directed=True, connection="strong")[0] == 1
    ids, ds, ctr, gh = oracle.search(ix, Q, k=t, l=t, T=0, entry=entry, t_seeds=t, want_ghost=True, **kw)
    for i in range(len(Q)):
        top, nodes, dn = _ghost_expect(X, Q[i], gmap, t)
        assert gh[i].tolist() == top.tolist()
        assert ids[i].tolist() == nodes.tolist()
        assert np.array_equal(ds[i], dn)
        assert not np.array_equal(ids[i], np.sort(top))  # ghost indices are not node ids here


# ---------------------------------------------------------------------------
# Similarity-threshold pruning (Sec. 6.3): instead of the fixed top-n of the
# direction ranking, a filtered expansion keeps every slot whose sign mismatch
# is at most floor(theta d); the parent is partly expanded only if a slot was
# skipped.
# ---------------------------------------------------------------------------
def test_threshold_one_keeps_every_slot_and_equals_plain_search():
    X = small(600, 16, C=5)
    Q = small(30, 16, C=5, seed=2)
    ix = oracle.build_index(X, deg=10, dgs=True)
    plain = oracle.search(ix, Q, k=10, l=32, T=50)
    o = oracle.search(ix, Q, k=10, l=32, T=50, dgs_on=True, dgs_threshold=1.0)
    assert np.array_equal(plain[0], o[0]) and np.array_equal(plain[1], o[1])
    assert np.array_equal(plain[2][:, :3], o[2][:, :3]) and np.all(o[2][:, 3] == 0)


def test_threshold_on_a_line_keeps_all_aligned_slots():
    """The chain of the cool-down pin with node 0 -> (1, 2), both toward the query. With d = 1 and
    theta = 0.999 the threshold is floor(0.999) = 0 mismatches: node 0 keeps both slots (top-n with
    n = 1 would keep one), node i keeps i + 1 and skips i - 1. T = 9, c = 0.3: 6 filtered iterations
    expand 0, 2, 3, 4, 5, 6 (five of them skip one slot), the cool-down expands 7, 8, 9."""
    n = 12
    G = [[1, 2]] + [[i - 1, i + 1] for i in range(1, n - 1)] + [[n - 2, n - 3]]
    X, ix = _line_index(range(n), np.array(G))
    q = np.array([[20.0]], np.float32)
    ids, ds, ctr = oracle.search(ix, q, k=3, l=n, T=9, entry="seeds", seeds=np.array([[0]]), dgs_on=True,
                                 dgs_threshold=0.999, cooldown=0.3)
    assert ids[0].tolist() == [10, 9, 8]
    assert ctr[0, 3] == 5 and ctr[0, 1] == 9 and ctr[0, 0] == 11


def test_threshold_skipping_every_slot_leaves_the_parent_partial():
    """In 2-D, a parent whose two neighbours both point away from the query on both axes keeps neither
    (theta = 0.5: at most one mismatch of two); it stays partial and the cool-down expands it in full."""
    X = np.array([[0.0, 0.0], [-1.0, -1.0], [-2.0, -1.5], [5.0, 5.0]], np.float32)
    G = np.array([[1, 2], [0, 2], [0, 1], [0, 1]])
    X, ix = np.asarray(X), oracle.build_index(X, deg=2, dgs=True, graph=G)
    q = np.array([[4.0, 4.0]], np.float32)
    ids, ds, ctr = oracle.search(ix, q, k=3, l=4, T=3, entry="seeds", seeds=np.array([[0]]), dgs_on=True,
                                 dgs_threshold=0.5, cooldown=0.3)
    # it 0 (filtered): node 0 skips both slots; no fresh entry is left, so the cool-down starts and
    # it 1 expands node 0 in full (1 and 2 found); it 2 expands node 1 (nothing new)
    assert ids[0].tolist() == [0, 1, 2]
    assert ctr[0, 3] == 2 and ctr[0, 1] == 3 and ctr[0, 0] == 3 and ctr[0, 2] == 3
    with pytest.raises(ValueError):
        oracle.search(ix, q, k=3, l=4, T=3, dgs_on=True, dgs_threshold=0.5, random_discard=True)


# ---------------------------------------------------------------------------
# Dynamic updates (Sec. 6.2): deletion flags and insertion into a shard.
# ---------------------------------------------------------------------------
def test_deleted_nodes_are_never_returned_exhaustive_search_is_brute_force_over_live():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((250, 10)).astype(np.float32)
    Q = rng.standard_normal((20, 10)).astype(np.float32)
    ix = oracle.build_index(X, deg=10, dgs=True)
    base = oracle.search(ix, Q, k=10, l=250, T=300)
    dead = rng.choice(250, 60, replace=False)
    oracle.delete(ix, dead)
    ids, ds, ctr = oracle.search(ix, Q, k=10, l=250, T=300)
    _, D = oracle.brute_force_numpy(X, Q, 10)
    D[:, dead] = np.inf
    assert np.array_equal(ids, f32_order(D, 10))
    assert not np.isin(ids, dead).any()
    # the traversal itself is unchanged: the same nodes are evaluated and expanded
    assert np.array_equal(base[2], ctr)
    # no flag set: identical to an index without flags
    ix.shards[0]["dead"][:] = 0
    again = oracle.search(ix, Q, k=10, l=250, T=300)
    assert np.array_equal(again[0], base[0]) and np.array_equal(again[1], base[1])


def test_deleted_node_still_bridges_and_low_precision_reranks_live_entries():
    """A line 0 - 1 - 2 - 3 with the query beside node 3 and the search seeded at node 0: node 1, deleted,
    is the only way on, and the search still reaches 2 and 3 through it; the result skips 1."""
    G = np.array([[1, 1], [0, 2], [1, 3], [2, 2]])
    X, ix = _line_index([0.0, 1.0, 2.0, 3.0], G)
    oracle.delete(ix, [1])
    ids, ds, ctr = oracle.search(ix, np.array([[3.2]], np.float32), k=3, l=4, T=10, entry="seeds",
                                 seeds=np.array([[0]]))
    assert ids[0].tolist() == [3, 2, 0]
    Xf = small(300, 32, C=3)
    Q = small(10, 32, C=3, seed=2)
    for store in ("f16", "fp8"):
        lp = oracle.build_index(Xf, deg=10, dgs=False, store=store)
        full = oracle.search(lp, Q, k=5, l=40, T=60)
        oracle.delete(lp, full[0][:, 0])  # every query's best result
        ids, ds, ctr = oracle.search(lp, Q, k=5, l=40, T=60)
        assert not np.isin(ids, full[0][:, 0]).any()
        assert np.all(ctr[:, 6] == 20)  # the rerank takes the first 4k live entries


def test_append_to_one_shard_equals_building_from_all_rows():
    X = small(500, 16, C=4)
    ixa = oracle.build_index(X[:420], deg=8, dgs=True, ghost_R=40, deg_g=8)
    oracle.append(ixa, 0, X[420:], ghost_seed=5)
    ixb = oracle.build_index(X, deg=8, dgs=True, ghost_R=40, deg_g=8)
    a, b = ixa.shards[0], ixb.shards[0]
    for key in ("graph", "sign", "gmap", "g_map", "g_graph"):
        assert np.array_equal(a[key], b[key]), key
    Q = small(30, 16, C=4, seed=2)
    for kw in (dict(dgs_on=True), dict(entry="ghost_graph"), dict(entry="ghost_dense", dgs_on=True)):
        ra = oracle.search(ixa, Q, k=10, l=32, T=40, **kw)
        rb = oracle.search(ixb, Q, k=10, l=32, T=40, **kw)
        assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])


def test_append_keeps_inter_shard_maps_exact():
    X = small(600, 12, C=3)
    ix = oracle.build_index(X, deg=8, S=3, dgs=False)
    new = small(50, 12, C=3, seed=7)
    oracle.append(ix, 1, new)
    assert ix.shards[1]["n"] == 250 and ix.n_total == 650
    assert np.array_equal(ix.shards[1]["gmap"][-50:], np.arange(600, 650))
    for s in range(3):
        A = ix.shards[s]["orig_base"]
        B = ix.shards[(s + 1) % 3]["orig_base"]
        _, D = oracle.brute_force_numpy(B, A, 1)
        assert np.array_equal(ix.shards[s]["next"], f32_order(D, 1)[:, 0])
    # the appended rows are found by their new global ids
    ids, _, _ = oracle.search(ix, new[:5], k=1, l=64, T=80, n_init=32)
    assert ids[:, 0].tolist() == list(range(600, 605))


# ---------------------------------------------------------------------------
# The lookup table built by search (Sec. 4): every node of a shard searches the adjacent shard, top-1 kept
# ---------------------------------------------------------------------------
def test_search_built_lookup_table_exhaustive_equals_exact_nearest():
    """An exhaustive search (queue longer than the shard, T beyond it) on a connected graph reaches the whole
    shard, so its top-1 is the brute-force nearest node: the search-built table equals I(u) of Sec. 3.1.2."""
    X = small(500, 12, C=1, sigma=1.0, seed=21)
    ix = oracle.build_index(X, deg=12, S=2, dgs=True)
    for s in range(2):
        nx = ix.shards[(s + 1) % 2]
        A = csr_matrix((np.ones(nx["graph"].size), nx["graph"].ravel(),
                        np.arange(0, nx["graph"].size + 1, nx["graph"].shape[1])), shape=(nx["n"], nx["n"]))
        assert connected_components(A, directed=True, connection="strong")[0] == 1
        lut = oracle.next_map_by_search(ix, s, l=nx["n"], T=2 * nx["n"], n_init=8)
        _, D = oracle.brute_force_numpy(nx["orig_base"], ix.shards[s]["orig_base"], 1)
        assert np.array_equal(lut, f32_order(D, 1)[:, 0])
        assert np.array_equal(lut, ix.shards[s]["next"])


def test_search_built_lookup_table_is_the_per_node_search():
    """Entry u is the top-1 local id of one search of node u on the next shard alone, keyed by u: the same
    value as a 1-shard index of that shard searched with the node as its only query."""
    X = small(600, 16, C=3, seed=22)
    ix = oracle.build_index(X, deg=8, S=3, dgs=True, ghost_R=30, deg_g=8)
    kw = dict(l=16, T=6, entry="ghost_graph", dgs_on=True)
    lut = oracle.next_map_by_search(ix, 1, **kw)
    nx = ix.shards[2]
    assert lut.max() < nx["n"]
    one = oracle.OracleIndex(dtype=ix.dtype, d=ix.d, deg=ix.deg, S=1, n_total=nx["n"], deg_g=ix.deg_g)
    sh = dict(nx)
    sh.pop("next")
    sh["gmap"] = np.arange(nx["n"], dtype=np.uint32)
    one.shards.append(sh)
    src = ix.shards[1]["orig_base"]
    for u in (0, 17, 150, len(src) - 1):
        ids, _, _ = oracle.search(one, src[u:u + 1], qkeys=np.array([u], np.uint64), k=1, **kw)
        assert lut[u] == ids[0, 0]
    # a short search does not always find the nearest node; where it does not, its pick is farther
    _, D = oracle.brute_force_numpy(nx["orig_base"], src, nx["n"])
    exact = f32_order(D, 1)[:, 0]
    miss = lut != exact
    assert 0 < miss.mean() < 0.5
    d32 = D.astype(np.float32)
    rows = np.arange(len(src))
    assert np.all(d32[rows[miss], lut[miss]] >= d32[rows[miss], exact[miss]])
