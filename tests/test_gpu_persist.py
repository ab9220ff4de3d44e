"""GPU round trip of miann_index_save / miann_index_load: the loaded index holds
the same arrays and returns the same ids, distances and counters as the saved one."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import d2h, dev, say, to_device_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")


def _same_arrays(a, b):
    ia, ib = a.info(), b.info()
    assert ia == ib
    for s in range(ia["num_shards"]):
        va, vb = a.shard(s), b.shard(s)
        assert (va.n, va.n_ghost, va.degree, va.ghost_degree, va.in_dtype) == \
            (vb.n, vb.n_ghost, vb.degree, vb.ghost_degree, vb.in_dtype)
        assert np.array_equal(d2h(va.graph, va.n * va.degree, np.uint32), d2h(vb.graph, vb.n * vb.degree, np.uint32))
        if va.n_ghost:
            assert np.array_equal(d2h(va.ghost_ids, va.n_ghost, np.uint32), d2h(vb.ghost_ids, vb.n_ghost, np.uint32))


def _same_search(a, b, Q, opts, itopk=64, T=60):
    qd = dev(Q)
    ra = a.search(qd, 10, itopk, T, opts, counters=True)
    rb = b.search(qd, 10, itopk, T, opts, counters=True)
    torch.cuda.synchronize()
    for x, y in zip(ra, rb):
        assert torch.equal(x, y)


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_save_load_imported_index(tmp_path, store):
    """Two shards with path extension and ghost shards, imported from the oracle's build."""
    say(f"save/load imported index store={store}")
    X = synth.mixture_small(2000, 96, 8, 0.25, 61)
    Q = synth.mixture_small(120, 96, 8, 0.25, 62)
    ox = oracle.build_index(X, deg=32, S=2, dgs=True, store=store, ghost_ratio=0.05, deg_g=16)
    gx = to_device_index(ox)
    path = str(tmp_path / "idx.bin")
    gx.save(path)
    lx = miann.Index.load(path)
    _same_arrays(gx, lx)
    for kw in (dict(), dict(dgs=True, entry="ghost_dense"), dict(entry="ghost_graph", search_width=2)):
        _same_search(gx, lx, Q, miann.SearchOptions(**kw))


def test_save_load_device_built_u8(tmp_path):
    """A single-shard uint8 index built on the device (no global-id map, no ghosts)."""
    say("save/load device-built u8 index")
    X = synth.to_u8(synth.mixture_small(1500, 64, 8, 0.3, 71))
    Q = synth.to_u8(synth.mixture_small(100, 64, 8, 0.3, 72))
    gx = miann.Index.build(dev(X), degree=16, num_shards=1, dgs_table=True)
    path = str(tmp_path / "u8.bin")
    gx.save(path)
    lx = miann.Index.load(path)
    _same_arrays(gx, lx)
    _same_search(gx, lx, Q, miann.SearchOptions(dgs=True))
