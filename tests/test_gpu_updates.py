"""GPU parity of the dynamic updates (Sec. 6.2) against the CPU oracle.

Deletion flags: the same global ids are flagged on both sides; deleted nodes
are still traversed and handed over between shards, but no result returns
them (each stage keeps the live entries of its queue in order, and a
low-precision store reranks the first live ones).

Insertion into a shard: both sides append the same rows to one shard and
rebuild its graph, direction table, store, inter-shard maps and ghost shards.
The rebuilt arrays are compared with the oracle's (bit-exact for uint8 rows;
for float rows the k-NN graph rows agree on >= 99.9% of nodes, as in the
build parity tests), and the search over the appended index is compared with
the oracle's search over a copy of the device's arrays.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare, d2h, dev, oracle_from_device, run_both, say, to_device_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")


def u8rows(n, d, C, seed):
    return np.clip(np.rint(128 + 32 * synth.mixture_small(n, d, C, 0.3, seed)), 0, 255).astype(np.uint8)


DEL_CASES = [
    ("plain", "f32", 10, 64, 60, dict()),
    ("dgs_dense", "f32", 10, 64, 40, dict(dgs=True, entry="ghost_dense", search_width=2)),
    ("graph_every_stage", "f32", 10, 48, 40, dict(dgs=True, entry="ghost_graph", ghost_every_stage=True)),
    ("f16_rerank", "f16", 10, 64, 40, dict(dgs=True, entry="ghost_dense")),
    ("fp8_k20", "fp8", 20, 128, 40, dict(dgs=True)),
]


@pytest.fixture(scope="module")
def deleted():
    X = synth.mixture_small(5000, 96, 10, 0.25, 151)
    Q = synth.mixture_small(300, 96, 10, 0.25, 152)
    rng = np.random.default_rng(153)
    gone = rng.choice(5000, 700, replace=False).astype(np.uint32)
    # the queries' own nearest neighbours are among the deleted ones, so deletions change the results
    gt, _ = oracle.knn(X, Q[:100], 3)
    gone = np.unique(np.concatenate([gone, gt.ravel().astype(np.uint32)]))
    idx = {}
    for store in ("f32", "f16", "fp8"):
        ox = oracle.build_index(X, deg=32, S=3, dgs=True, store=store, ghost_ratio=0.04, deg_g=16)
        gx = to_device_index(ox)
        oracle.delete(ox, gone)
        gx.delete(dev(gone))
        idx[store] = (ox, gx)
    return Q, gone, idx


@pytest.mark.parametrize("name,store,k,itopk,T,kw", DEL_CASES, ids=[c[0] for c in DEL_CASES])
def test_deletion_flags_parity(deleted, name, store, k, itopk, T, kw):
    Q, gone, idx = deleted
    ox, gx = idx[store]
    say(f"deletion flags case={name} store={store} deleted={len(gone)}")
    opts = miann.SearchOptions(**kw)
    g, o = run_both(ox, gx, Q, k, itopk, T, opts)
    compare(g, o, label=f"del-{name}", ndist_check=False)
    got = g[0]
    assert not np.isin(got[got != 0xFFFFFFFF], gone).any()


def test_deletion_flags_accumulate():
    """A second call adds flags; ids outside the index are ignored."""
    X = synth.mixture_small(2000, 32, 4, 0.25, 161)
    ox = oracle.build_index(X, deg=16)
    gx = to_device_index(ox)
    a, b = np.arange(0, 2000, 7, dtype=np.uint32), np.array([3, 5, 1 << 29], np.uint32)
    for part in (a, b):
        oracle.delete(ox, part)
        gx.delete(dev(part))
    Qs = synth.mixture_small(100, 32, 4, 0.25, 162)
    g, o = run_both(ox, gx, Qs, 10, 64, 40, miann.SearchOptions())
    compare(g, o, label="del-accumulate", ndist_check=False)
    assert not np.isin(g[0], np.concatenate([a, b[:2]])).any()


def shard_arrays(gx, s):
    v = gx.shard(s)
    out = dict(n=v.n, gmap=d2h(v.global_ids, v.n, np.uint32),
               graph=d2h(v.graph, v.n * v.degree, np.uint32).reshape(v.n, v.degree))
    if v.next_map:
        out["next"] = d2h(v.next_map, v.n, np.uint32)
    if v.n_ghost:
        out["g_map"] = d2h(v.ghost_ids, v.n_ghost, np.uint32)
    return out


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_append_rebuilds_the_shard(dtype):
    n0, n_new, d = 4000, 600, 64
    if dtype == "u8":
        X = u8rows(n0 + n_new, d, 8, 171)
        Q = u8rows(200, d, 8, 172)
    else:
        X = synth.mixture_small(n0 + n_new, d, 8, 0.3, 171)
        Q = synth.mixture_small(200, d, 8, 0.3, 172)
    ox = oracle.build_index(X[:n0], deg=32, S=3, dgs=True, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    # a deletion before the insertion: the flags of the old rows survive the rebuild
    gone = np.arange(0, n0, 11, dtype=np.uint32)
    oracle.delete(ox, gone)
    gx.delete(dev(gone))
    s = 1
    say(f"append {n_new} {dtype} rows to shard {s} of 3")
    oracle.append(ox, s, X[n0:], ghost_seed=5)
    gx.append(s, dev(X[n0:]), ghost_seed=5)
    info = gx.info()
    assert info["n"] == n0 + n_new
    for t in range(3):
        G, O = shard_arrays(gx, t), ox.shards[t]
        assert G["n"] == O["n"]
        assert np.array_equal(G["gmap"], O["gmap"])
        same = np.all(G["graph"] == O["graph"], axis=1)
        say(f"  shard {t}: graph rows identical {same.mean():.4f}, next map identical "
            f"{np.mean(G['next'] == O['next']):.4f}, ghosts identical {np.array_equal(G['g_map'], O['g_map'])}")
        assert np.array_equal(G["g_map"], O["g_map"])
        if dtype == "u8":
            assert same.all() and np.array_equal(G["next"], O["next"])
        else:
            assert same.mean() >= 0.999 and np.mean(G["next"] == O["next"]) >= 0.999
    # the search over the appended index, against the oracle on the device's own arrays and flags
    ox2 = oracle_from_device(gx, X)
    oracle.delete(ox2, gone)
    for name, kw in (("plain", dict()), ("dgs_dense", dict(dgs=True, entry="ghost_dense", search_width=2))):
        opts = miann.SearchOptions(**kw)
        g, o = run_both(ox2, gx, Q, 10, 64, 40, opts)
        compare(g, o, label=f"append-{dtype}-{name}", ndist_check=False)
        found = g[0][g[0] != 0xFFFFFFFF]
        assert not np.isin(found, gone).any()
    # the new rows are reachable: each is its own nearest neighbour
    qn = X[n0:n0 + 50]
    g, o = run_both(ox2, gx, qn, 1, 64, 60, miann.SearchOptions(entry="ghost_dense"))
    assert np.mean(g[0][:, 0] == np.arange(n0, n0 + 50)) >= 0.95
