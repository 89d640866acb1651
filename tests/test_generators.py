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


def test_planted_partition_structure():
    n, groups, f_in = 1 << 14, 32, 0.8
    g = gg.planted(n, groups, avg_degree=16, f_in=f_in, seed=3)
    T.check_canonical(g)
    h = gg.planted(n, groups, avg_degree=16, f_in=f_in, seed=3)
    assert np.array_equal(g.adjncy, h.adjncy)
    deg = np.diff(g.xadj.astype(np.int64))
    src = np.repeat(np.arange(n), deg)
    same = (src * groups // n) == (g.adjncy.astype(np.int64) * groups // n)
    # a draw lands inside its group with probability f_in + (1 - f_in) / groups
    want = f_in + (1 - f_in) / groups
    assert abs(same.mean() - want) < 0.01
    assert abs(deg.mean() - 16) < 0.5  # few duplicates at this density


def test_chung_lu_degrees_follow_weights():
    n, d, gamma = 1 << 14, 16.0, 2.5
    g = gg.chung_lu(n, avg_degree=d, gamma=gamma, seed=4)
    T.check_canonical(g)
    deg = np.diff(g.xadj.astype(np.int64))
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1 / (gamma - 1))
    expected = 2 * (d * n / 2) * w / w.sum()  # two endpoint draws per edge
    # low-degree nodes: mean degree close to the expected weight
    tail = slice(n // 2, n)
    assert abs(deg[tail].mean() - expected[tail].mean()) < 0.15 * expected[tail].mean()
    # heavy head (duplicates merge there), decreasing on average
    assert deg[:16].mean() > 10 * deg.mean()
    assert deg[: n // 16].mean() > deg[n // 16: n // 4].mean() > deg[n // 4:].mean()
