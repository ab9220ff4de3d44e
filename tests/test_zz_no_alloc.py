"""The search entry point that allocates nothing (miann_search_noalloc), called
through the C-ABI: on two calls in a row, the second with a smaller batch, it
returns exactly what miann_search returns on the same inputs (the same
kernels run on buffers carved from the library's static device array), with
four resident shards and the dense ghost entry on every stage (hand-off,
per-stage results and the dense entry's work area all live in that array).
Batches that do not fit the array are rejected before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, say, to_device_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")


@pytest.fixture(scope="module")
def sharded():
    X = synth.mixture_small(6000, 96, 12, 0.25, 131)
    Q = synth.mixture_small(700, 96, 12, 0.25, 132)
    ox = oracle.build_index(X, deg=32, S=4, dgs=True, ghost_ratio=0.03, deg_g=16)
    return Q, ox, to_device_index(ox)


def call(gx, fn, Q, k, itopk, T, opts):
    """Calls the C entry point `fn` with caller-allocated outputs; returns host ids and dists."""
    nq = Q.shape[0]
    qd = dev(Q)
    ids = torch.full((nq, k), -7, dtype=torch.int32, device="cuda")
    dists = torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda")
    ctr = torch.zeros((nq, miann.NCTR), dtype=torch.int64, device="cuda")
    p = opts.cstruct()
    rc = fn(gx.handle, qd.data_ptr(), nq, k, itopk, T, ctypes.byref(p), ids.data_ptr(), dists.data_ptr(),
            ctr.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0, miann.load().miann_last_error()
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), dists.cpu().numpy(), ctr.cpu().numpy()


CASES = [
    ("dense_every_stage", 10, 64, 24, dict(entry="ghost_dense", dgs=True, search_width=2, ghost_every_stage=True,
                                           t_seeds=8)),
    ("dense_start_only", 10, 64, 24, dict(entry="ghost_dense", dgs=True)),
    ("graph_entry", 10, 48, 24, dict(entry="ghost_graph", dgs=True)),
]


@pytest.mark.parametrize("name,k,itopk,T,kw", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_search_on_two_calls(sharded, name, k, itopk, T, kw):
    Q, ox, gx = sharded
    L = miann.load()
    opts = miann.SearchOptions(**kw)
    for n in (700, 213):  # the second call smaller: the array keeps the first call's contents
        say(f"noalloc case={name} nq={n} k={k} itopk={itopk} T={T}")
        ref = call(gx, L.miann_search, Q[:n], k, itopk, T, opts)
        got = call(gx, L.miann_search_noalloc, Q[:n], k, itopk, T, opts)
        assert np.array_equal(got[0], ref[0]), name
        assert np.array_equal(got[1].view(np.uint32), ref[1].view(np.uint32)), name
        assert np.array_equal(got[2], ref[2]), name
        # and the oracle agrees with both on this shape (the bar of the other parity tests)
        oi = oracle.search(ox, Q[:n], k=k, l=itopk, r=opts.search_width, T=T, entry=opts.entry,
                           t_seeds=opts.t_seeds or None, dgs_on=opts.dgs,
                           ghost_every_stage=opts.ghost_every_stage)[0]
        assert np.mean(np.all(got[0] == oi, axis=1)) >= 0.999


def test_noalloc_rejects_what_does_not_fit(sharded):
    Q, ox, gx = sharded
    L = miann.load()
    cap = L.miann_noalloc_scratch_bytes()
    assert cap == miann.load().miann_noalloc_scratch_bytes() > 0
    # 4 shards x k = 512 keys of 8 bytes per query: 16 KB per query, so cap / 8 KB queries cannot fit
    nq = cap // 8192 + 64
    opts = miann.SearchOptions(entry="ghost_dense", ghost_every_stage=True)
    p = opts.cstruct()
    q = torch.zeros((nq, 96), dtype=torch.float32, device="cuda")
    ids = torch.empty((nq, 512), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, 512), dtype=torch.float32, device="cuda")
    rc = L.miann_search_noalloc(gx.handle, q.data_ptr(), nq, 512, 512, 8, ctypes.byref(p), ids.data_ptr(),
                                dists.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    assert rc == 1 and b"scratch" in L.miann_last_error()
    # timing into phase_ms would create events: rejected too
    tb = (ctypes.c_float * 6)()
    p.phase_ms = ctypes.cast(tb, ctypes.c_void_p)
    rc = L.miann_search_noalloc(gx.handle, q.data_ptr(), 8, 10, 64, 8, ctypes.byref(p), ids.data_ptr(),
                                dists.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    assert rc == 1 and b"phase_ms" in L.miann_last_error()
