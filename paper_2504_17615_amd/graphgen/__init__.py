"""Seeded synthetic inputs shaped like the paper's graph classes.

This module only synthesises graphs (Appendix C lists the paper's classes:
meshes as the local control, R-MAT, Erdos-Renyi and geometric graphs as the
non-local / weighted cases).  It contains none of the partitioning method's
arithmetic and is the one module shared by the GPU library's tests and
benchmark and by the CPU oracle's tests.

Graphs are returned as :class:`Graph` holding a canonical symmetric CSR
(numpy arrays): ``xadj`` uint64[n+1], ``adjncy`` uint32[M] with sorted rows,
no self-loops and no duplicates; ``adjwgt`` int32[M] or ``None`` (unit);
``vwgt`` is always ``None`` (unit node weights).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from paper_2504_17615_amd.build import build_graphgen

        build_graphgen()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, u32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
    lib.gg_grid.argtypes = [u64, u64]
    lib.gg_grid.restype = vp
    lib.gg_rmat.argtypes = [u32, u64, dbl, dbl, dbl, u64]
    lib.gg_rmat.restype = vp
    lib.gg_er.argtypes = [u64, u64, u64]
    lib.gg_er.restype = vp
    lib.gg_rgg.argtypes = [u64, dbl, u64]
    lib.gg_rgg.restype = vp
    lib.gg_planted.argtypes = [u64, u64, dbl, dbl, u64]
    lib.gg_planted.restype = vp
    lib.gg_chung_lu.argtypes = [u64, dbl, dbl, u64]
    lib.gg_chung_lu.restype = vp
    lib.gg_n.argtypes = [vp]
    lib.gg_n.restype = u64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_nnz.restype = u64
    lib.gg_weighted.argtypes = [vp]
    lib.gg_weighted.restype = ctypes.c_int
    lib.gg_copy.argtypes = [vp, vp, vp, vp]
    lib.gg_copy.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_free.restype = None
    _lib = lib
    return lib


@dataclass
class Graph:
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: Optional[np.ndarray] = None
    vwgt: Optional[np.ndarray] = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.adjncy.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2


def _collect(h, name) -> Graph:
    lib = _load()
    try:
        n = int(lib.gg_n(h))
        nnz = int(lib.gg_nnz(h))
        xadj = np.empty(n + 1, dtype=np.uint64)
        adj = np.empty(nnz, dtype=np.uint32)
        w = np.empty(nnz, dtype=np.int32) if lib.gg_weighted(h) else None
        lib.gg_copy(h, xadj.ctypes.data, adj.ctypes.data, None if w is None else w.ctypes.data)
    finally:
        lib.gg_free(h)
    return Graph(n=n, xadj=xadj, adjncy=adj, adjwgt=w, name=name)


def grid(rows: int, cols: int) -> Graph:
    return _collect(_load().gg_grid(rows, cols), f"grid{rows}x{cols}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 22) -> Graph:
    return _collect(_load().gg_rmat(scale, edge_factor, a, b, c, seed), f"rmat{scale}")


def er(n: int, m: int, seed: int = 23) -> Graph:
    if m > n * (n - 1) // 2:
        raise ValueError("more edges than pairs")
    return _collect(_load().gg_er(n, m, seed), f"er{n}_{m}")


def rgg_radius(n: int, avg_degree: float = 12.0) -> float:
    # expected degree of a point away from the border is pi r^2 n
    return math.sqrt(avg_degree / (math.pi * n))


def rgg(n: int, r: Optional[float] = None, seed: int = 24) -> Graph:
    if r is None:
        r = rgg_radius(n)
    return _collect(_load().gg_rgg(n, r, seed), f"rgg{n}")


def planted(n: int, groups: int, avg_degree: float = 32.0, f_in: float = 0.8,
            seed: int = 25) -> Graph:
    """Planted partition: n nodes in `groups` contiguous groups, a fraction
    f_in of the edge draws inside a group."""
    return _collect(_load().gg_planted(n, groups, avg_degree, f_in, seed), f"planted{n}_{groups}")


def chung_lu(n: int, avg_degree: float = 32.0, gamma: float = 2.5, seed: int = 26) -> Graph:
    """Chung-Lu graph with power-law expected degrees (exponent gamma)."""
    return _collect(_load().gg_chung_lu(n, avg_degree, gamma, seed), f"chunglu{n}")


# The workloads: (graph factory, k, eps, seed).  Full sizes plus reduced
# shapes of the same recipes that the CPU oracle finishes in seconds.
def workload(name: str):
    """Return (graph, k, eps, seed) for a named workload."""
    if name == "grid128":
        return grid(128, 128), 4, 0.03, 1
    if name == "rmat22":
        return rmat(22), 64, 0.03, 1
    if name == "er22":
        return er(1 << 22, 1 << 26), 128, 0.03, 1
    if name == "rgg24":
        return rgg(1 << 24), 256, 0.03, 1
    # reduced shapes (same recipes)
    if name.startswith("rmat"):
        s = int(name[4:])
        return rmat(s), 64, 0.03, 1
    if name.startswith("er"):
        s = int(name[2:])
        return er(1 << s, 1 << (s + 4)), 128, 0.03, 1
    if name.startswith("rgg"):
        s = int(name[3:])
        return rgg(1 << s), 256, 0.03, 1
    if name.startswith("grid"):
        s = int(name[4:])
        return grid(s, s), 4, 0.03, 1
    raise KeyError(name)


def _mix64(x: int) -> int:
    """SplitMix64 step (Steele, Lea, Flood, OOPSLA 2014): the request mix's
    counter-based draws."""
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return x ^ (x >> 31)


def request_spec(i: int, lo_exp: float, hi_exp: float):
    """Request i of the serving mix: (kind, n, k) with n = floor(10^(lo + (hi -
    lo) u)) nodes (u uniform), kind 0 grid (rows = floor(sqrt n), cols = ceil(n /
    rows)), 1 R-MAT (edge factor 16, scale round(log2 n)), 2 Erdos-Renyi
    G(n, 16n); k = 2 (1 + H mod 128); eps 0.03 and seed i + 1 go with it."""
    u = (_mix64(3 * i) >> 11) / float(1 << 53)
    n = int(10 ** (lo_exp + (hi_exp - lo_exp) * u))
    kind = _mix64(3 * i + 1) % 3
    k = 2 * (1 + _mix64(3 * i + 2) % 128)
    return kind, n, k


def request_graph(i: int, lo_exp: float, hi_exp: float):
    """(graph, k, eps, seed) of request i of the serving mix."""
    kind, n, k = request_spec(i, lo_exp, hi_exp)
    if kind == 0:
        rows = max(2, int(n ** 0.5))
        g = grid(rows, -(-n // rows))
    elif kind == 1:
        g = rmat(max(4, int(round(float(np.log2(n))))), seed=i + 1)
    else:
        g = er(n, 16 * n, seed=i + 1)
    return g, min(k, g.n), 0.03, i + 1


def request_mix(n_req: int, lo_exp: float, hi_exp: float, threads: int = 1, first: int = 0):
    """Requests first .. first + n_req - 1 of the serving mix, generated on
    `threads` threads (the generator releases the interpreter lock)."""
    ids = range(first, first + n_req)
    if threads <= 1:
        return [request_graph(i, lo_exp, hi_exp) for i in ids]
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda i: request_graph(i, lo_exp, hi_exp), ids))
