"""Small hand-made graphs for tests (test helper; no partitioning arithmetic)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class G:
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: Optional[np.ndarray] = None
    vwgt: Optional[np.ndarray] = None

    @property
    def nnz(self):
        return int(self.adjncy.shape[0])

    @property
    def m(self):
        return self.nnz // 2


def from_edges(n, edges, weights=None, vwgt=None) -> G:
    """Canonical symmetric CSR from undirected edges {u, v} (u != v, no repeats)."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if weights is None:
        w = None
    else:
        w = np.asarray(weights, dtype=np.int64)
    src = np.concatenate([edges[:, 0], edges[:, 1]])
    dst = np.concatenate([edges[:, 1], edges[:, 0]])
    ww = None if w is None else np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    if ww is not None:
        ww = ww[order]
    assert np.all(src != dst), "self-loop"
    if len(src) > 1:
        dup = (src[1:] == src[:-1]) & (dst[1:] == dst[:-1])
        assert not dup.any(), "duplicate edge"
    xadj = np.zeros(n + 1, np.uint64)
    np.add.at(xadj, src + 1, 1)
    xadj = np.cumsum(xadj).astype(np.uint64)
    return G(n, xadj, dst.astype(np.uint32), None if ww is None else ww.astype(np.int64),
             None if vwgt is None else np.asarray(vwgt, np.int64))


def star(leaves):
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def path(n):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def two_cliques(s):
    e = [(a, b) for a in range(s) for b in range(a + 1, s)]
    e += [(a + s, b + s) for a, b in e]
    return from_edges(2 * s, e)


def random_graph(n, m, rng, wmax=1, vmax=1, connected_chain=False):
    pairs = set()
    if connected_chain:
        for i in range(n - 1):
            pairs.add((i, i + 1))
    while len(pairs) < m:
        u, v = rng.integers(0, n, size=2)
        if u == v:
            continue
        pairs.add((min(u, v), max(u, v)))
    e = sorted(pairs)
    w = rng.integers(1, wmax + 1, size=len(e)) if wmax > 1 else None
    vw = rng.integers(1, vmax + 1, size=n) if vmax > 1 else None
    return from_edges(n, e, w, vw)


def edges_of(g):
    """Undirected edges (a < b) with weights, from a CSR."""
    deg = np.diff(g.xadj.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = g.adjncy.astype(np.int64)
    w = (np.ones(len(dst), np.int64) if g.adjwgt is None
         else np.asarray(g.adjwgt, np.int64))
    sel = src < dst
    return src[sel], dst[sel], w[sel]


def node_weights(g):
    return np.ones(g.n, np.int64) if g.vwgt is None else np.asarray(g.vwgt, np.int64)


def check_canonical(g):
    """Symmetric, sorted rows, no self-loops, no duplicates, positive weights."""
    xadj = g.xadj.astype(np.int64)
    assert xadj[0] == 0 and np.all(np.diff(xadj) >= 0)
    deg = np.diff(xadj)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = g.adjncy.astype(np.int64)
    assert np.all(dst < g.n)
    assert np.all(src != dst), "self-loop"
    key = src * g.n + dst
    assert np.all(np.diff(key) > 0), "rows not sorted / duplicates"
    rkey = dst * g.n + src
    order = np.argsort(rkey)
    assert np.array_equal(rkey[order], key), "not symmetric"
    if g.adjwgt is not None:
        w = np.asarray(g.adjwgt, np.int64)
        assert np.all(w > 0)
        assert np.array_equal(w[order], w), "asymmetric weights"
