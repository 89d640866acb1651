"""Seeded input generators: shapes, canonical form, determinism."""
import numpy as np

from paper_2504_17615_amd import graphgen as gg
from tests import graphs as T


def test_grid_shape():
    g = gg.grid(128, 128)
    assert g.n == 16384 and g.m == 32512 and g.nnz == 65024
    T.check_canonical(g)
    deg = np.diff(g.xadj.astype(np.int64))
    assert sorted(set(deg.tolist())) == [2, 3, 4]
    assert int((deg == 2).sum()) == 4


def test_rmat_canonical_and_deterministic():
    a = gg.rmat(12, seed=7)
    b = gg.rmat(12, seed=7)
    c = gg.rmat(12, seed=8)
    assert a.n == 4096
    T.check_canonical(a)
    assert np.array_equal(a.adjncy, b.adjncy) and np.array_equal(a.xadj, b.xadj)
    assert not np.array_equal(a.adjncy, c.adjncy)
    # skew: quadrant a=0.57 puts the heaviest rows at small ids
    deg = np.diff(a.xadj.astype(np.int64))
    assert deg[:64].mean() > 4 * deg.mean()


def test_er_exact_edge_count():
    g = gg.er(1 << 12, 1 << 15, seed=3)
    assert g.n == 4096 and g.m == 1 << 15
    T.check_canonical(g)


def test_rgg_weights_and_degree():
    g = gg.rgg(1 << 14, seed=5)
    T.check_canonical(g)
    assert g.adjwgt is not None
    assert g.adjwgt.min() >= 1 and g.adjwgt.max() <= 9
    avg = g.nnz / g.n
    assert 10 < avg < 12.5  # pi r^2 n = 12 minus border losses


def test_workload_table():
    g, k, eps, seed = gg.workload("grid128")
    assert (k, eps, seed) == (4, 0.03, 1)
    g, k, eps, seed = gg.workload("rmat12")
    assert k == 64 and g.n == 4096
