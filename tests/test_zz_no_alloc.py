"""The allocation-free entry point (lmgp_partition_noalloc) against
lmgp_partition: identical blocks, cut, balance and level count, on calls in a
row (the second on a smaller graph, so the scratch array holds the previous
call's contents), for device and host outputs, at the size limit, and the
rejection of a graph above the limit."""
import ctypes

import numpy as np
import pytest

from paper_2504_17615_amd import graphgen as gg
from tests import graphs as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_17615_amd as L

    L.library()
    return L


FIELDS = ("cut", "max_block_weight", "lmax", "levels")


def _both(L, g, k, seed, host):
    print(f"noalloc n={g.n} nnz={g.nnz} k={k} seed={seed} host={host}", flush=True)
    dg = L.create_graph(g)
    want, wres = dg.partition(k, 0.03, seed, host_out=True)
    if host:
        before = torch.cuda.memory_allocated()
        got, gres = dg.partition(k, 0.03, seed, host_out=True, noalloc=True)
        assert torch.cuda.memory_allocated() == before
    else:
        out = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        _, gres = dg.partition(k, 0.03, seed, out=out, noalloc=True)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    for f in FIELDS:
        assert gres[f] == wres[f], (f, gres[f], wres[f])
    dg.close()


def test_noalloc_calls_in_a_row(lib):
    # a larger graph, then a smaller one (scratch keeps the larger call's data)
    _both(lib, gg.rmat(16), 64, 1, host=False)
    _both(lib, gg.grid(48, 48), 4, 2, host=False)
    _both(lib, gg.er(1 << 14, 1 << 17, seed=3), 16, 3, host=True)
    _both(lib, T.from_edges(9, [(0, 1), (1, 2)]), 2, 4, host=True)  # isolated nodes


def test_noalloc_at_the_size_limit(lib):
    n, nnz = lib.NOALLOC_MAX_NODES, lib.NOALLOC_MAX_ENTRIES
    g = gg.er(n, nnz // 2, seed=5)  # n = 2^19 nodes, 2^22 entries
    assert g.n == n and g.nnz == nnz
    _both(lib, g, 128, 5, host=False)
    g = gg.rmat(17)  # power-law degrees below the entry limit
    assert g.nnz <= nnz
    _both(lib, g, 64, 6, host=False)


def test_noalloc_rejects_too_large_graphs(lib):
    n = lib.NOALLOC_MAX_NODES + 1
    g = T.G(n, np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32))
    dg = lib.create_graph(g)
    out = np.empty(n, np.uint32)
    from paper_2504_17615_amd._binding import Result

    res = Result()
    api = lib.library()
    st = api.lmgp_partition_noalloc(dg.handle, 2, 0.03, 1, None,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    out.ctypes.data, 0, ctypes.byref(res))
    assert st == 1  # LMGP_EINVAL
    assert b"too large" in api.lmgp_last_error()
    dg.close()
