"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer graph work, so the bar is bit-exact equality: every hierarchy level
(CSR, node and edge weights, fine-to-coarse map, level statistics), the final
block of every node, the cut, the maximum block weight and L_max.
"""
import numpy as np
import pytest

import oracle as O
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


INFO_KEYS = ("n", "m", "m_prime", "m_hat", "triggered", "lp_rounds", "twohop", "w_t", "n_gt",
             "n_eq", "nclusters_lp")


def check_hierarchy(L, g, k, seed, **kw):
    print(f"hierarchy n={g.n} m={g.nnz // 2} k={k} seed={seed} {kw}", flush=True)
    dg = L.create_graph(g, validate=True)
    h = dg.coarsen(k, seed, L.default_params(**kw))
    oh = O.coarsen(g, k, seed, O.params(**kw))
    assert h.levels == len(oh.levels)
    for i in range(h.levels):
        got, want = h.info(i), oh.info[i]
        for key in INFO_KEYS:
            assert got[key] == want[key], (i, key, got[key], want[key])
        lv = h.copy_level(i)
        ol = oh.levels[i]
        assert np.array_equal(lv["xadj"], ol.xadj), i
        assert np.array_equal(lv["adjncy"], ol.adjncy), i
        assert np.array_equal(lv["vwgt"], ol.vwgt), i
        assert np.array_equal(lv["adjwgt"], ol.adjwgt), i
        if i + 1 < h.levels:
            assert np.array_equal(lv["map"], oh.maps[i]), i
    h.close()
    dg.close()
    return oh


def check_partition(L, g, k, eps, seed, **kw):
    print(f"partition n={g.n} m={g.nnz // 2} k={k} eps={eps} seed={seed} {kw}", flush=True)
    dg = L.create_graph(g)
    blocks, res = dg.partition(k, eps, seed, L.default_params(**kw), host_out=True)
    ob, ores, _ = O.partition(g, k, eps, seed, O.params(**kw))
    assert res["cut"] == ores["cut"]
    assert res["max_block_weight"] == ores["max_block_weight"]
    assert res["lmax"] == ores["lmax"]
    assert res["levels"] == ores["levels"]
    assert np.array_equal(blocks, ob)
    # device output path gives the same bytes
    dblocks, _ = dg.partition(k, eps, seed, L.default_params(**kw))
    assert np.array_equal(dblocks.cpu().numpy().view(np.uint32), ob)
    dg.close()
    return res


SMALL = ["grid128", "rmat12", "rmat14", "er12", "er14", "rgg14", "rgg16"]


@pytest.mark.parametrize("name", SMALL)
def test_hierarchy_parity(lib, name):
    g, k, eps, seed = gg.workload(name)
    check_hierarchy(lib, g, min(k, 16), seed)


@pytest.mark.parametrize("name", SMALL)
def test_partition_parity(lib, name):
    g, k, eps, seed = gg.workload(name)
    check_partition(lib, g, k, eps, seed)


@pytest.mark.parametrize("name", ["rmat16", "er16", "rgg18"])
def test_partition_parity_mid(lib, name):
    g, k, eps, seed = gg.workload(name)
    check_partition(lib, g, k, eps, seed)


@pytest.mark.parametrize("seed", range(4))
def test_weighted_random_graphs(lib, seed):
    rng = np.random.default_rng(seed)
    g = T.random_graph(3000, 20000, rng, wmax=9, vmax=5)
    check_hierarchy(lib, g, 4, seed)
    check_partition(lib, g, 4, 0.05, seed)


@pytest.mark.parametrize("subrounds", [1, 32])
def test_subround_counts(lib, subrounds):
    # 32 sub-rounds x 13 degree classes: the largest bucket histogram
    g, k, eps, seed = gg.workload("rmat14")
    check_hierarchy(lib, g, 16, seed, subrounds=subrounds)
    check_partition(lib, g, k, eps, seed, subrounds=subrounds)


@pytest.mark.parametrize("sampler", [1, 3])
@pytest.mark.parametrize("name", ["er14", "rmat14"])
def test_sparsification_samplers(lib, name, sampler):
    # uniform random sampling and threshold sampling with coins for E^=
    g, k, eps, seed = gg.workload(name)
    check_hierarchy(lib, g, 16, seed, sampler=sampler)
    check_partition(lib, g, k, eps, seed, sampler=sampler)


@pytest.mark.parametrize("cap", ["1", "64"])
@pytest.mark.parametrize("name", ["er14", "rmat14"])
def test_eq_rank_scan_path(lib, name, cap, monkeypatch):
    # the rank inside E^= with a gather buffer too small for the selected
    # bucket: the rank kernel scans the edge range itself (same result)
    g, k, eps, seed = gg.workload(name)
    monkeypatch.setenv("LMGP_EQ_GATHER_CAP", cap)
    oh = check_hierarchy(lib, g, 16, seed, sampler=0)
    ranked = [i for i in oh.info if i["triggered"] and i["m_hat"] - i["n_gt"] != i["n_eq"]]
    assert ranked, "no level ranks inside E^="
    check_partition(lib, g, k, eps, seed, sampler=0)


def test_sparsification_off(lib):
    g, k, eps, seed = gg.workload("er14")
    check_hierarchy(lib, g, 16, seed, sampler=2)
    check_partition(lib, g, k, eps, seed, sampler=2)


@pytest.mark.parametrize("leaves", [5000, 7000, 12000])
def test_hub_rows(lib, leaves):
    # stars exercise the big-node rating classes (8192- and 16384-slot tables,
    # global tables) and the 1024-thread LDS contraction rows (8192- and
    # 16384-word classes)
    g = T.star(leaves)
    check_hierarchy(lib, g, 2, 3)
    check_partition(lib, g, 2, 0.03, 3)


@pytest.mark.parametrize("tables", ["ranges", "global", "repair"])
def test_hub_rating_paths(lib, tables, monkeypatch):
    # degree 20000 > 8192: label-range LDS rating, forced global tables, or
    # every range recomputed by the overflow repair passes
    if tables != "ranges":
        monkeypatch.setenv("LMGP_HUB_TABLES", tables)
    rng = np.random.default_rng(9)
    s = T.star(20000)
    a, b, _ = T.edges_of(s)
    extra = set()
    while len(extra) < 30000:  # leaves also linked among themselves
        x, y = rng.integers(1, s.n, size=2)
        if x != y:
            extra.add((min(x, y), max(x, y)))
    e = np.concatenate([np.stack([a, b], 1), np.array(sorted(extra))])
    g = T.from_edges(s.n, e)
    check_hierarchy(lib, g, 4, 3)
    check_partition(lib, g, 4, 0.03, 3)


@pytest.mark.parametrize("mode", ["ranges", "overflow"])
def test_large_contraction_rows(lib, mode, monkeypatch):
    # coarse rows of more than 12288 entries: hash ranges in LDS, or the
    # radix-sorted rows that replace them when a range does not fit
    if mode == "overflow":
        monkeypatch.setenv("LMGP_ROW_RANGES", "overflow")
    rng = np.random.default_rng(4)
    s = T.star(30000)
    a, b, _ = T.edges_of(s)
    extra = set()
    while len(extra) < 60000:
        x, y = rng.integers(1, s.n, size=2)
        if x != y:
            extra.add((min(x, y), max(x, y)))
    g = T.from_edges(s.n, np.concatenate([np.stack([a, b], 1), np.array(sorted(extra))]))
    check_hierarchy(lib, g, 4, 5)
    check_partition(lib, g, 4, 0.03, 5)


def test_hub_rows_heavy_weights(lib):
    # total edge weight >= 2^32 switches the hub and big-node rating tables
    # from packed 64-bit slots to separate key / 64-bit value arrays
    s = T.star(12000)
    rng = np.random.default_rng(5)
    a, b, _ = T.edges_of(s)
    w = rng.integers(1 << 19, 1 << 20, size=len(a))
    g = T.from_edges(s.n, np.stack([a, b], 1), w)
    assert int(g.adjwgt.sum()) >= 1 << 32
    check_hierarchy(lib, g, 2, 3)
    check_partition(lib, g, 2, 0.03, 3)


def test_packed_wide_coarse_weights(lib):
    # 2^31 <= total edge weight < 2^32: ratings still fit 32 bits (packed
    # tables, 32-bit dense rows) while coarse weights stay int64
    rng = np.random.default_rng(12)
    g = T.random_graph(3000, 20000, rng)
    w = rng.integers(50000, 60000, size=g.nnz // 2)
    a, b, _ = T.edges_of(g)
    g = T.from_edges(g.n, np.stack([a, b], 1), w)
    assert (1 << 31) <= int(g.adjwgt.sum()) < (1 << 32)
    check_hierarchy(lib, g, 8, 6)
    check_partition(lib, g, 8, 0.03, 6)


def test_dense_rows_heavy_weights(lib):
    # total edge weight >= 2^32: refinement's dense rows (one wave per node,
    # 256-thread rows) keep 64-bit counters instead of 32-bit ones
    rng = np.random.default_rng(8)
    n = 4000
    edges = set()
    while len(edges) < 20000:
        a, b = (int(x) for x in rng.integers(n, size=2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    for h, d in zip(range(20), np.linspace(150, 3000, 20).astype(int)):
        for b in rng.choice(n, size=d, replace=False):
            if int(b) != h:
                edges.add((min(h, int(b)), max(h, int(b))))
    e = np.array(sorted(edges))
    w = rng.integers(1 << 19, 1 << 20, size=len(e))
    g = T.from_edges(n, e, w)
    assert int(g.adjwgt.sum()) >= 1 << 32
    check_partition(lib, g, 8, 0.03, 4)


def _shuffle_rows(g, rng):
    adj = g.adjncy.copy()
    w = None if g.adjwgt is None else g.adjwgt.copy()
    for u in range(g.n):
        a, b = int(g.xadj[u]), int(g.xadj[u + 1])
        perm = rng.permutation(b - a) + a
        adj[a:b] = g.adjncy[perm]
        if w is not None:
            w[a:b] = g.adjwgt[perm]
    return T.G(g.n, g.xadj.copy(), adj, w, g.vwgt)


@pytest.mark.parametrize("n", [300, 5000])
def test_unsorted_input_rows(lib, n):
    # rows in arbitrary order (accepted without full validation): the
    # breadth-first bisection visits neighbours in the given row order, which
    # the oracle follows too; n = 300 with k = 2 partitions the input level
    # itself, n = 5000 coarsens first (coarse rows are built sorted)
    rng = np.random.default_rng(n)
    g = _shuffle_rows(T.random_graph(n, 6 * n, rng, wmax=5, vmax=3), rng)
    print(f"unsorted rows n={n}", flush=True)
    dg = lib.create_graph(g)
    blocks, res = dg.partition(2, 0.03, 7, host_out=True)
    ob, ores, _ = O.partition(g, 2, 0.03, 7)
    assert np.array_equal(blocks, ob)
    assert res["cut"] == ores["cut"]
    dg.close()


def test_tiny_and_degenerate(lib):
    check_partition(lib, T.path(2), 2, 0.03, 1)
    check_partition(lib, T.from_edges(5, [(0, 1)]), 3, 0.03, 1)  # isolated nodes
    check_partition(lib, T.two_cliques(8), 2, 0.03, 3)
    check_partition(lib, gg.grid(40, 40), 1, 0.03, 1)
    g = T.from_edges(400, [])  # no edges at all
    check_partition(lib, g, 4, 0.03, 2)
