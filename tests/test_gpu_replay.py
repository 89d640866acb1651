"""LP rounds captured into a HIP graph and replayed (lmgp_params.graph_rounds).

Replayed rounds launch with upper-bound grids and take their counts from a
plan written on the device; the result must be byte-identical to the oracle's
(and so to the round-by-round launches), alone, in a batch and together with
the autotuned class tables.
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


def case(name):
    if name == "star7000":  # a node in the 16384-slot class (packed ratings)
        return T.star(7000), 2, 0.03, 3
    if name == "weighted":
        rng = np.random.default_rng(7)
        return T.random_graph(3000, 40000, rng, wmax=9, vmax=5), 8, 0.05, 7
    if name == "rmat14_k2000":  # hashed refinement tables (more than 1024 blocks)
        g, _, eps, seed = gg.workload("rmat14")
        return g, 2000, eps, seed
    return gg.workload(name)


@pytest.mark.parametrize("name", ["grid128", "rmat12", "rmat14", "er14", "rgg14", "rgg16",
                                  "star7000", "weighted", "rmat14_k2000"])
def test_replayed_rounds_match_oracle(lib, name):
    g, k, eps, seed = case(name)
    print(f"replayed rounds on {name}: n={g.n} m={g.nnz // 2} k={k}", flush=True)
    dg = lib.create_graph(g)
    prm = lib.default_params(graph_rounds=1)
    blocks, res = dg.partition(k, eps, seed, prm, host_out=True)
    ob, ores, _ = O.partition(g, k, eps, seed, O.params())
    assert res["cut"] == ores["cut"]
    assert res["max_block_weight"] == ores["max_block_weight"]
    assert res["levels"] == ores["levels"]
    assert np.array_equal(blocks, ob)
    # the hierarchy (clustering rounds replayed too) level by level
    h = dg.coarsen(k, seed, prm)
    oh = O.coarsen(g, k, seed, O.params())
    assert h.levels == len(oh.levels)
    for i in range(h.levels):
        assert h.info(i)["lp_rounds"] == oh.info[i]["lp_rounds"], i
        assert h.info(i)["nclusters_lp"] == oh.info[i]["nclusters_lp"], i
        lv = h.copy_level(i)
        assert np.array_equal(lv["adjncy"], oh.levels[i].adjncy), i
    h.close()
    dg.close()


def test_replayed_rounds_in_a_batch(lib):
    # graphs of uneven size share each replayed round; some stop before others
    gs = [gg.workload("grid128")[0], gg.workload("rmat12")[0], gg.workload("er12")[0],
          T.star(3000)]
    ks, seeds = [4, 16, 8, 2], [1, 2, 3, 4]
    dgs = [lib.create_graph(g) for g in gs]
    print("replayed rounds in a batch of 4", flush=True)
    outs, res = lib.partition_batch(dgs, ks, [0.03] * 4, seeds, lib.default_params(graph_rounds=1))
    for i, g in enumerate(gs):
        ob, ores, _ = O.partition(g, ks[i], 0.03, seeds[i], O.params())
        assert res[i]["cut"] == ores["cut"], i
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint32), ob), i
    for d in dgs:
        d.close()


def test_replay_with_autotuned_tables(lib):
    g, k, eps, seed = gg.workload("rmat16")
    print("replayed rounds with autotuned tables on rmat16", flush=True)
    dg = lib.create_graph(g)
    want, _ = dg.partition(k, eps, seed, lib.default_params(), host_out=True)
    got, _ = dg.partition(k, eps, seed, lib.default_params(graph_rounds=1, tune=1), host_out=True)
    assert np.array_equal(got, want)
    dg.close()
