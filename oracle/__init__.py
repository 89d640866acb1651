"""Python access to the CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never imports it.  It imports
nothing from the GPU library.  Graph arguments are duck-typed: any object with
``n``, ``xadj`` (uint64), ``adjncy`` (uint32) and optional ``vwgt`` /
``adjwgt`` (any integer dtype, converted to int64 here) works.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TAGS = dict(SUB=1, TIE=2, ADM=3, FAV=4, TWOHOP=5, SPARS=6, IP=7, RSUB=8, RTIE=9, RADM=10,
            FFSTART=11, FFDRAW=12, FFBREAK=13, FFCLAIM=14)


class Params(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_uint32) for nm in (
        "tau_e_num", "tau_e_den", "tau_d_num", "tau_d_den", "rho_num", "rho_den", "sampler",
        "clim", "shrink_num", "shrink_den", "lp_rounds", "ref_rounds", "subrounds",
        "max_levels", "stop_num", "stop_den", "ff_p_num", "ff_p_den", "ff_nu_num",
        "ff_nu_den")]


class CGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("m_prime", ctypes.c_uint64),
                ("m_hat", ctypes.c_uint64), ("triggered", ctypes.c_uint32),
                ("lp_rounds", ctypes.c_uint32), ("twohop", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("w_t", ctypes.c_int64), ("n_gt", ctypes.c_uint64),
                ("n_eq", ctypes.c_uint64), ("nclusters_lp", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "pad"}


class Result(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("max_block_weight", ctypes.c_int64),
                ("lmax", ctypes.c_int64), ("levels", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle.build import build

        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u64, u32, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64
    sig = {
        "or_set_threads": ([ctypes.c_int], ctypes.c_int),
        "or_hash": ([u64, u64, u32, vp], u64),
        "or_mix": ([u64], u64),
        "or_default_params": ([vp], None),
        "or_graph_new": ([vp], vp),
        "or_free": ([vp], None),
        "or_g_n": ([vp], u64),
        "or_g_nnz": ([vp], u64),
        "or_g_copy": ([vp, vp, vp, vp, vp], None),
        "or_cluster": ([vp, i64, u64, u64, vp, vp, vp], None),
        "or_label_propagation": ([vp, vp, vp, u64, i64, u64, u64, u32, u32, u32, u32, vp], u32),
        "or_fire_scores": ([vp, u64, u64, u32, u32, u32, u32, u32, vp, vp], None),
        "or_contract": ([vp, vp, vp], vp),
        "or_edge_budget": ([u64, u64, u64, vp], u64),
        "or_budget_triggers": ([u64, u64, vp], ctypes.c_int),
        "or_sparsify": ([vp, u64, u64, u64, u32, vp, vp], vp),
        "or_coarsen": ([vp, u32, u64, vp], vp),
        "or_h_levels": ([vp], u32),
        "or_h_info": ([vp, u32, vp], None),
        "or_h_n": ([vp, u32], u64),
        "or_h_nnz": ([vp, u32], u64),
        "or_h_copy": ([vp, u32, vp, vp, vp, vp, vp], None),
        "or_initial_partition": ([vp, u32, u64, u64, vp], None),
        "or_refine": ([vp, vp, u32, i64, u64, u64, vp], u64),
        "or_balance_limit": ([i64, u32, ctypes.c_double], i64),
        "or_evaluate": ([vp, vp, u32, vp, vp], None),
        "or_partition": ([vp, u32, ctypes.c_double, u64, vp, vp, vp, vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


@dataclass
class OGraph:
    """A graph produced by the oracle (int64 weights, always materialised)."""
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    vwgt: np.ndarray
    adjwgt: np.ndarray

    @property
    def nnz(self):
        return int(self.adjncy.shape[0])

    @property
    def m(self):
        return self.nnz // 2


class _View:
    """Keeps int64 copies alive while a CGraph points at them."""

    def __init__(self, g):
        self.n = int(g.n)
        self.xadj = np.ascontiguousarray(g.xadj, dtype=np.uint64)
        self.adjncy = np.ascontiguousarray(g.adjncy, dtype=np.uint32)
        vw = getattr(g, "vwgt", None)
        ew = getattr(g, "adjwgt", None)
        self.vwgt = None if vw is None else np.ascontiguousarray(vw, dtype=np.int64)
        self.adjwgt = None if ew is None else np.ascontiguousarray(ew, dtype=np.int64)
        self.c = CGraph(self.n, self.xadj.ctypes.data, self.adjncy.ctypes.data,
                        None if self.vwgt is None else self.vwgt.ctypes.data,
                        None if self.adjwgt is None else self.adjwgt.ctypes.data)

    @property
    def ref(self):
        return ctypes.byref(self.c)


def params(**kw) -> Params:
    p = Params()
    _load().or_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel steps (1 = single-threaded, the
    default); returns the number in effect."""
    return int(_load().or_set_threads(int(n)))


def H(seed: int, tag: int, *xs: int) -> int:
    arr = (ctypes.c_uint64 * max(1, len(xs)))(*[x & (2**64 - 1) for x in xs])
    return int(_load().or_hash(seed & (2**64 - 1), tag, len(xs), arr))


def mix(z: int) -> int:
    return int(_load().or_mix(z & (2**64 - 1)))


def _take_graph(h) -> OGraph:
    lib = _load()
    try:
        n = int(lib.or_g_n(h))
        nnz = int(lib.or_g_nnz(h))
        xadj = np.empty(n + 1, np.uint64)
        adj = np.empty(nnz, np.uint32)
        vw = np.empty(n, np.int64)
        ew = np.empty(nnz, np.int64)
        lib.or_g_copy(h, xadj.ctypes.data, adj.ctypes.data, vw.ctypes.data, ew.ctypes.data)
    finally:
        lib.or_free(h)
    return OGraph(n, xadj, adj, vw, ew)


def normalise(g) -> OGraph:
    """The oracle's own canonical copy of a graph (int64 weights)."""
    v = _View(g)
    return _take_graph(_load().or_graph_new(v.ref))


def cluster(g, U: int, seed: int, level: int, p: Optional[Params] = None):
    p = p or params()
    v = _View(g)
    lab = np.empty(v.n, np.uint32)
    st = np.zeros(4, np.uint64)
    _load().or_cluster(v.ref, U, seed, level, ctypes.byref(p), lab.ctypes.data, st.ctypes.data)
    return lab, dict(lp_rounds=int(st[0]), nclusters_lp=int(st[1]), twohop=int(st[2]),
                     nclusters=int(st[3]))


def label_propagation(g, label, W, cap, seed, level, refine_tags=False, rounds=5, subrounds=4,
                      shrink_stop=False):
    v = _View(g)
    lab = np.ascontiguousarray(label, np.uint32).copy()
    w = np.ascontiguousarray(W, np.int64).copy()
    moves = ctypes.c_uint64(0)
    r = _load().or_label_propagation(v.ref, lab.ctypes.data, w.ctypes.data, w.shape[0], cap, seed,
                                     level, int(refine_tags), rounds, subrounds, int(shrink_stop),
                                     ctypes.byref(moves))
    return lab, w, int(r), int(moves.value)


def fire_scores(g, seed, level, weighted=True, p=(3, 5), nu=(1, 2)):
    """(Weighted) Forest Fire burn score of every entry; returns (scores,
    dict(fires=..., burns=...))."""
    if not all(0 <= x < 1 << 32 for x in (*p, *nu)):
        raise ValueError("fire parameters are 32-bit rationals")
    v = _View(g)
    sc = np.empty(v.adjncy.shape[0], np.int64)
    st = np.zeros(2, np.uint64)
    _load().or_fire_scores(v.ref, seed, level, int(weighted), p[0], p[1], nu[0], nu[1],
                           sc.ctypes.data, st.ctypes.data)
    return sc, dict(fires=int(st[0]), burns=int(st[1]))


def contract(g, label):
    v = _View(g)
    lab = np.ascontiguousarray(label, np.uint32)
    mp = np.empty(v.n, np.uint32)
    h = _load().or_contract(v.ref, lab.ctypes.data, mp.ctypes.data)
    return _take_graph(h), mp


def edge_budget(m, n, n_next, p: Optional[Params] = None) -> int:
    p = p or params()
    return int(_load().or_edge_budget(m, n, n_next, ctypes.byref(p)))


def budget_triggers(m_prime, m_hat, p: Optional[Params] = None) -> bool:
    p = p or params()
    return bool(_load().or_budget_triggers(m_prime, m_hat, ctypes.byref(p)))


def sparsify(g, m_hat, seed, level, sampler=0, p: Optional[Params] = None):
    """sampler 0: exact-size threshold sampling, 1: uniform random sampling,
    3: threshold sampling with independent coins for the edges of weight w_t,
    4 / 5: exact-size threshold sampling on (Weighted) Forest Fire scores
    (fire parameters from p, defaults if None)."""
    v = _View(g)
    st = np.zeros(3, np.int64)
    h = _load().or_sparsify(v.ref, m_hat, seed, level, sampler,
                            ctypes.byref(p) if p is not None else None, st.ctypes.data)
    return _take_graph(h), dict(w_t=int(st[0]), n_gt=int(st[1]), n_eq=int(st[2]))


@dataclass
class Hierarchy:
    levels: List[OGraph] = field(default_factory=list)
    maps: List[np.ndarray] = field(default_factory=list)
    info: List[dict] = field(default_factory=list)


def coarsen(g, k, seed, p: Optional[Params] = None) -> Hierarchy:
    p = p or params()
    lib = _load()
    v = _View(g)
    h = lib.or_coarsen(v.ref, k, seed, ctypes.byref(p))
    out = Hierarchy()
    try:
        L = int(lib.or_h_levels(h))
        for lvl in range(L):
            n = int(lib.or_h_n(h, lvl))
            nnz = int(lib.or_h_nnz(h, lvl))
            xadj = np.empty(n + 1, np.uint64)
            adj = np.empty(nnz, np.uint32)
            vw = np.empty(n, np.int64)
            ew = np.empty(nnz, np.int64)
            mp = np.empty(n, np.uint32) if lvl + 1 < L else None
            lib.or_h_copy(h, lvl, xadj.ctypes.data, adj.ctypes.data, vw.ctypes.data,
                          ew.ctypes.data, None if mp is None else mp.ctypes.data)
            out.levels.append(OGraph(n, xadj, adj, vw, ew))
            if mp is not None:
                out.maps.append(mp)
            li = LevelInfo()
            lib.or_h_info(h, lvl, ctypes.byref(li))
            out.info.append(li.as_dict())
    finally:
        lib.or_free(h)
    return out


def initial_partition(g, k, seed, level):
    v = _View(g)
    b = np.empty(v.n, np.uint32)
    _load().or_initial_partition(v.ref, k, seed, level, b.ctypes.data)
    return b


def refine(g, block, k, lmax, seed, level, p: Optional[Params] = None):
    p = p or params()
    v = _View(g)
    b = np.ascontiguousarray(block, np.uint32).copy()
    moves = _load().or_refine(v.ref, b.ctypes.data, k, lmax, seed, level, ctypes.byref(p))
    return b, int(moves)


def balance_limit(cV, k, eps) -> int:
    return int(_load().or_balance_limit(cV, k, eps))


def evaluate(g, block, k):
    v = _View(g)
    b = np.ascontiguousarray(block, np.uint32)
    cut = ctypes.c_int64()
    mx = ctypes.c_int64()
    _load().or_evaluate(v.ref, b.ctypes.data, k, ctypes.byref(cut), ctypes.byref(mx))
    return int(cut.value), int(mx.value)


def partition(g, k, eps, seed, p: Optional[Params] = None):
    """Returns (block, result dict, phase times in seconds)."""
    p = p or params()
    v = _View(g)
    b = np.empty(v.n, np.uint32)
    res = Result()
    t = np.zeros(3, np.int64)
    _load().or_partition(v.ref, k, eps, seed, ctypes.byref(p), b.ctypes.data, ctypes.byref(res),
                         t.ctypes.data)
    r = dict(cut=int(res.cut), max_block_weight=int(res.max_block_weight), lmax=int(res.lmax),
             levels=int(res.levels))
    times = dict(coarsen=t[0] * 1e-9, initial=t[1] * 1e-9, refine=t[2] * 1e-9)
    return b, r, times
