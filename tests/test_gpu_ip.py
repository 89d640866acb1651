"""Initial partitioning on the device (lmgp_params.ip_device = 1).

The recursive bisection by greedy growing runs one workgroup per subproblem
and dequeues whole frontiers at once; it must give the host rule's blocks
exactly, so every partition here is compared with the oracle byte for byte:
dense and sparse coarsest levels, isolated nodes, disconnected graphs, rows in
the caller's order, k from 1 to well above the coarsest level's size, and a
batch whose graphs end their hierarchies at different levels.
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


def _shuffle_rows(g, rng):
    adj = g.adjncy.copy()
    w = None if g.adjwgt is None else g.adjwgt.copy()
    for u in range(g.n):
        a, b = int(g.xadj[u]), int(g.xadj[u + 1])
        p = rng.permutation(b - a) + a
        adj[a:b] = g.adjncy[p]
        if w is not None:
            w[a:b] = g.adjwgt[p]
    return T.G(g.n, g.xadj.copy(), adj, w, g.vwgt)


def check(lib, g, k, eps, seed, ip=1, **kw):
    where = "device" if ip == 1 else "host"
    print(f"{where} IP: n={g.n} m={g.nnz // 2} k={k} seed={seed} {kw}", flush=True)
    dg = lib.create_graph(g)
    blocks, res = dg.partition(k, eps, seed, lib.default_params(ip_device=ip, **kw), host_out=True)
    ob, ores, _ = O.partition(g, k, eps, seed, O.params(**kw))
    assert res["cut"] == ores["cut"]
    assert res["max_block_weight"] == ores["max_block_weight"]
    assert res["levels"] == ores["levels"]
    assert np.array_equal(blocks, ob)
    dg.close()


@pytest.mark.parametrize("ip", [1, 0])
@pytest.mark.parametrize("name", ["grid128", "rmat12", "rmat14", "er12", "er14", "rgg14",
                                  "rgg16", "rmat16"])
def test_device_ip_workloads(lib, name, ip):
    g, k, eps, seed = gg.workload(name)
    check(lib, g, k, eps, seed, ip)


@pytest.mark.parametrize("k", [1, 2, 3, 7, 100, 2000])
def test_device_ip_block_counts(lib, k):
    # k = 2000 > 160k / 160: no coarsening, the input level is bisected
    g, _, eps, seed = gg.workload("rmat14")
    check(lib, g, k, eps, seed)


@pytest.mark.parametrize("seed", range(3))
def test_device_ip_weighted(lib, seed):
    rng = np.random.default_rng(100 + seed)
    g = T.random_graph(3000, 20000, rng, wmax=9, vmax=7)
    check(lib, g, 6, 0.05, seed)


def test_device_ip_sparsified_levels(lib):
    # sampling leaves isolated nodes in the coarse levels
    g, k, eps, seed = gg.workload("er14")
    check(lib, g, k, eps, seed, sampler=1)


@pytest.mark.parametrize("ip", [1, 0])
def test_device_ip_degenerate(lib, ip):
    check(lib, T.path(2), 2, 0.03, 1, ip)
    check(lib, T.from_edges(5, [(0, 1)]), 3, 0.03, 1, ip)  # isolated nodes
    check(lib, T.two_cliques(8), 2, 0.03, 3, ip)
    check(lib, T.from_edges(400, []), 4, 0.03, 2, ip)  # no edges at all
    check(lib, T.star(5000), 2, 0.03, 3, ip)
    check(lib, T.star(300), 16, 0.03, 3, ip)


def _core_with_stragglers(rng, core=220, pendants=60, isolated=120):
    # a clique whose rows are long, nodes of degree one hanging off it, and
    # isolated nodes: the searches keep a few unvisited nodes of short rows
    # for long (the host bisection then walks them instead of scanning rows)
    edges = [(a, b) for a in range(core) for b in range(a + 1, core)]
    for p in range(pendants):
        edges.append((int(rng.integers(core)), core + p))
    n = core + pendants + isolated
    vw = rng.integers(1, 6, size=n)
    return T.from_edges(n, edges, vwgt=vw)


@pytest.mark.parametrize("ip", [0, 1])
@pytest.mark.parametrize("k", [2, 5, 16])
def test_dense_core_with_stragglers(lib, k, ip):
    g = _core_with_stragglers(np.random.default_rng(40 + k))
    check(lib, g, k, 0.03, 11, ip)


def test_device_ip_unsorted_rows(lib):
    rng = np.random.default_rng(300)
    g = _shuffle_rows(T.random_graph(300, 1800, rng, wmax=5, vmax=3), rng)
    check(lib, g, 2, 0.03, 7)
    check(lib, g, 5, 0.03, 7)


def test_device_ip_batch(lib):
    # hierarchies of different depths: the graphs are bisected at different levels
    gs = [gg.workload("grid128")[0], gg.workload("rmat12")[0], T.star(3000),
          T.random_graph(500, 3000, np.random.default_rng(9), wmax=3, vmax=2)]
    ks, seeds = [4, 16, 2, 5], [1, 2, 3, 4]
    dgs = [lib.create_graph(g) for g in gs]
    print("device IP in a batch of 4", flush=True)
    outs, res = lib.partition_batch(dgs, ks, [0.03] * 4, seeds, lib.default_params(ip_device=1))
    for i, g in enumerate(gs):
        ob, ores, _ = O.partition(g, ks[i], 0.03, seeds[i], O.params())
        assert res[i]["cut"] == ores["cut"], i
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint32), ob), i
    for d in dgs:
        d.close()


def test_automatic_choice_in_a_large_batch(lib):
    # 20 graphs sharing their coarsest level: the default (automatic) choice
    # bisects them on the device; single calls use the host
    rng = np.random.default_rng(21)
    gs = [T.random_graph(800, 5000, rng, wmax=3, vmax=2) for _ in range(20)]
    dgs = [lib.create_graph(g) for g in gs]
    print("automatic IP choice in a batch of 20", flush=True)
    outs, res = lib.partition_batch(dgs, [8] * 20, [0.03] * 20, list(range(20)))
    for i, g in enumerate(gs):
        ob, ores, _ = O.partition(g, 8, 0.03, i, O.params())
        assert res[i]["cut"] == ores["cut"], i
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint32), ob), i
    for d in dgs:
        d.close()


def test_host_ip_wide_ids(lib):
    # more than 2^16 nodes at the bisected level: the host copy keeps 32-bit
    # neighbour ids (smaller levels travel as 16-bit local ids)
    g = gg.rmat(17)
    assert g.n > (1 << 16)
    check(lib, g, 1000, 0.03, 5, 0)  # k = 1000: 160 k >= n, no coarsening
