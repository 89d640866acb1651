"""Degree-class tables of the rating kernels and their autotuner.

Every table routes each degree to a kernel able to hold it, so the choice can
change the speed only: under every table, forced or picked by the tuner, the
partition must be byte-identical to the oracle's (which has no such notion).
"""
import numpy as np
import pytest

import oracle as O
from paper_2504_17615_amd import graphgen as gg
from tests import graphs as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# forced table indices wrap modulo the number of tables of each kind (five
# hashed, eight dense-row tables), so 0..7 covers every table of both kinds
NTABLES = 8
TUNE_AUTO, TUNE_FORCE = 1, 16


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_17615_amd as L

    L.library()
    return L


def case(name):
    if name == "rmat16":  # coarse levels with nodes in every class; 64 blocks: dense rows
        g, k, eps, seed = gg.workload("rmat16")
        return g, k, eps, seed
    if name == "rmat14_k2000":  # more than 1024 blocks: hashed refinement tables
        g, _, eps, seed = gg.workload("rmat14")
        return g, 2000, eps, seed
    if name == "star7000":  # one node in the 16384-slot class
        return T.star(7000), 2, 0.03, 3
    if name == "star12000":  # global tables by default, the 16384-slot class at load 3/4
        return T.star(12000), 2, 0.03, 3
    if name == "weighted":
        rng = np.random.default_rng(5)
        return T.random_graph(3000, 40000, rng, wmax=9, vmax=5), 8, 0.05, 5
    raise KeyError(name)


_oracle = {}


def oracle_partition(name, g, k, eps, seed):
    if name not in _oracle:
        _oracle[name] = O.partition(g, k, eps, seed, O.params())
    return _oracle[name]


@pytest.mark.parametrize("table", range(NTABLES))
@pytest.mark.parametrize("name", ["rmat16", "rmat14_k2000", "star7000", "star12000",
                                  "weighted"])
def test_forced_tables_match_oracle(lib, name, table):
    g, k, eps, seed = case(name)
    print(f"table {table} on {name}: n={g.n} m={g.nnz // 2} k={k}", flush=True)
    dg = lib.create_graph(g)
    blocks, res = dg.partition(k, eps, seed, lib.default_params(tune=TUNE_FORCE + table),
                               host_out=True)
    ob, ores, _ = oracle_partition(name, g, k, eps, seed)
    assert res["cut"] == ores["cut"]
    assert res["max_block_weight"] == ores["max_block_weight"]
    assert res["levels"] == ores["levels"]
    assert np.array_equal(blocks, ob)
    dg.close()


def test_autotune_times_once_and_matches_default(lib):
    # R-MAT scale 18: its first levels are large enough to be timed
    g, k, eps, seed = gg.workload("rmat18")
    print(f"autotune on rmat18: n={g.n} m={g.nnz // 2} k={k}", flush=True)
    dg = lib.create_graph(g)
    want, wres = dg.partition(k, eps, seed, lib.default_params(), host_out=True)
    lib.tuner_clear()
    got, res = dg.partition(k, eps, seed, lib.default_params(tune=TUNE_AUTO), host_out=True)
    info = lib.tuner_info()
    assert info["trials"] > 0 and info["entries"] > 0
    assert res["cut"] == wres["cut"]
    assert np.array_equal(got, want)
    # the same level signatures again: served from the cache, no new trials
    got2, _ = dg.partition(k, eps, seed, lib.default_params(tune=TUNE_AUTO), host_out=True)
    assert lib.tuner_info()["trials"] == info["trials"]
    assert np.array_equal(got2, want)
    dg.close()
