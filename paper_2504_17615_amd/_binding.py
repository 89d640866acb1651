"""ctypes binding of liblmgp.so: argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import threading
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmgp.so")

_lib = None
_lock = threading.Lock()

# Limits of lmgp_partition_noalloc (LMGP_NOALLOC_* in include/lmgp.h).
NOALLOC_SCRATCH_BYTES = 256 << 20
NOALLOC_MAX_NODES = 1 << 19
NOALLOC_MAX_ENTRIES = 1 << 22


class LmgpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lmgp status {status}: {msg}")
        self.status = status


# --------------------------------------------------------------- structs --
class Params(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_uint32) for nm in (
        "tau_e_num", "tau_e_den", "tau_d_num", "tau_d_den", "rho_num", "rho_den", "sampler",
        "clim", "shrink_num", "shrink_den", "lp_rounds", "ref_rounds", "subrounds",
        "max_levels", "stop_num", "stop_den", "tune", "graph_rounds", "ip_device",
        "ff_p_num", "ff_p_den", "ff_nu_num", "ff_nu_den")]


class CsrView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("nnz", ctypes.c_uint64), ("xadj", ctypes.c_void_p),
                ("adjncy", ctypes.c_void_p), ("vwgt", ctypes.c_void_p),
                ("adjwgt", ctypes.c_void_p), ("vwgt_bits", ctypes.c_uint32),
                ("adjwgt_bits", ctypes.c_uint32), ("on_device", ctypes.c_uint32),
                ("validate", ctypes.c_uint32)]


class Allocator(ctypes.Structure):
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", ALLOC), ("free", FREE)]


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
                ("lmax", ctypes.c_int64), ("levels", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("t_coarsen_ns", ctypes.c_int64), ("t_initial_ns", ctypes.c_int64),
                ("t_refine_ns", ctypes.c_int64), ("t_total_ns", ctypes.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "pad"}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("ip_device", ctypes.c_uint32), ("join_runs", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_uint64) for nm in (
        "completed", "failed", "runs", "max_run_requests", "retried_alone", "joined",
        "peak_resident_estimate", "peak_pool_bytes")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_SIGS = {
    "lmgp_default_params": ([ctypes.c_void_p], None),
    "lmgp_last_error": ([], ctypes.c_char_p),
    "lmgp_graph_create": ([ctypes.c_void_p] * 4, ctypes.c_int),
    "lmgp_graph_destroy": ([ctypes.c_void_p], None),
    "lmgp_graph_info": ([ctypes.c_void_p] * 4, ctypes.c_int),
    "lmgp_coarsen": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_hierarchy_levels": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_hierarchy_level_info": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p],
                                  ctypes.c_int),
    "lmgp_hierarchy_copy_level": ([ctypes.c_void_p, ctypes.c_uint32] + [ctypes.c_void_p] * 5,
                                  ctypes.c_int),
    "lmgp_hierarchy_destroy": ([ctypes.c_void_p], None),
    "lmgp_partition": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                        ctypes.c_void_p], ctypes.c_int),
    "lmgp_partition_noalloc": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int),
    "lmgp_fire_scores": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                          ctypes.c_void_p], ctypes.c_int),
    "lmgp_partition_batch": ([ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                             ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_create": ([ctypes.c_void_p] * 3, ctypes.c_int),
    "lmgp_server_submit": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_double,
                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_submit_params": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                   ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_stats_read": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_poll": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_wait": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "lmgp_server_destroy": ([ctypes.c_void_p], None),
    "lmgp_profile_enable": ([ctypes.c_uint32], ctypes.c_int),
    "lmgp_profile_read": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32],
                          ctypes.c_int),
    "lmgp_profile_filter": ([ctypes.c_char_p], ctypes.c_int),
    "lmgp_tuner_info": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "lmgp_tuner_clear": ([], None),
}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64),
                ("total_ns", ctypes.c_uint64), ("bytes", ctypes.c_uint64)]


def profile_enable(on: bool = True):
    _check(library().lmgp_profile_enable(1 if on else 0))


def profile_filter(kernel: Optional[str] = None):
    """Time only the launches of `kernel` (None: every profiled launch)."""
    _check(library().lmgp_profile_filter(kernel.encode() if kernel else None))


def profile_read(reset: bool = True) -> dict:
    """Per kernel family: launches, summed event time (ns), algorithmic bytes."""
    cnt = ctypes.c_uint32()
    _check(library().lmgp_profile_read(None, 0, ctypes.byref(cnt), 0))
    arr = (KernelStat * max(1, cnt.value))()
    _check(library().lmgp_profile_read(arr, cnt.value, ctypes.byref(cnt), 1 if reset else 0))
    return {arr[i].name.decode(): dict(launches=int(arr[i].launches),
                                       total_ns=int(arr[i].total_ns), bytes=int(arr[i].bytes))
            for i in range(cnt.value)}

def tuner_info() -> dict:
    """The autotuner's process-wide cache: cached entries and timed trials."""
    e, t = ctypes.c_uint64(), ctypes.c_uint64()
    _check(library().lmgp_tuner_info(ctypes.byref(e), ctypes.byref(t)))
    return {"entries": int(e.value), "trials": int(t.value)}


def tuner_clear():
    library().lmgp_tuner_clear()


EXPORTED = tuple(_SIGS)


def library():
    """Load liblmgp.so (raises if it was not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2504_17615_amd.build lib`")
        # One HIP runtime per process: PyTorch loads its own copy of the
        # runtime by another file name, which would come in as a second
        # runtime (seeing no device) if it were loaded after this library's.
        # Loaded first, it also serves this library (same soname).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
        return lib


def _check(status: int):
    if status != 0:
        msg = library().lmgp_last_error()
        raise LmgpError(status, msg.decode() if msg else "")


def default_params(**overrides) -> Params:
    p = Params()
    library().lmgp_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _torch():
    import torch

    return torch


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        torch = _torch()
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator, for the library."""

    def __init__(self, device: int):
        torch = _torch()
        self.device = device

        def _alloc(ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                          int(stream or 0))
            except Exception:  # noqa: BLE001 - report NULL to the library
                return None

        def _free(ctx, ptr, stream):
            torch.cuda.caching_allocator_delete(ptr)

        self._a = Allocator.ALLOC(_alloc)
        self._f = Allocator.FREE(_free)
        self.struct = Allocator(None, self._a, self._f)


def _ptr(a):
    if a is None:
        return None, 0
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), a.element_size() * 8
    arr = np.ascontiguousarray(a)
    return arr.ctypes.data, arr.dtype.itemsize * 8


class DeviceGraph:
    """A validated graph resident in device memory (owns an lmgp_graph)."""

    def __init__(self, handle, n, nnz, keep=None, allocator=None):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.nnz = nnz
        self._keep = keep
        self._alloc = allocator

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            library().lmgp_graph_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def total_weight(self) -> int:
        n, nnz, tw = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64()
        _check(library().lmgp_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                         ctypes.byref(tw)))
        return int(tw.value)

    def partition(self, k: int, eps: float = 0.03, seed: int = 1, params: Optional[Params] = None,
                  stream=None, out=None, host_out: bool = False, noalloc: bool = False):
        """Returns (blocks, result dict).  blocks is a torch uint32-compatible
        int32 tensor on the device (or a numpy uint32 array if host_out).
        noalloc=True calls lmgp_partition_noalloc (the library's fixed scratch
        array instead of any allocation; `out` or host_out avoid torch's)."""
        res = Result()
        if host_out:
            blocks = np.empty(self.n, np.uint32)
            ptr, on_dev = blocks.ctypes.data, 0
        else:
            torch = _torch()
            blocks = out if out is not None else torch.empty(self.n, dtype=torch.int32,
                                                             device="cuda")
            ptr, on_dev = blocks.data_ptr(), 1
        fn = library().lmgp_partition_noalloc if noalloc else library().lmgp_partition
        _check(fn(self._h, k, eps, seed, ctypes.byref(params) if params is not None else None,
                  _stream_ptr(stream), ptr, on_dev, ctypes.byref(res)))
        return blocks, res.as_dict()

    def fire_scores(self, seed: int, level: int, weighted: bool = True,
                    params: Optional[Params] = None, stream=None, out=None,
                    host_out: bool = False):
        """(Weighted) Forest Fire burn score of every entry (lmgp_fire_scores).
        Returns (scores, dict(fires=, burns=, steps=)); scores is an int32
        torch tensor on the device (bit pattern of the uint32 scores) or a
        numpy uint32 array if host_out."""
        if host_out:
            sc = np.empty(max(self.nnz, 1), np.uint32)
            ptr, on_dev = sc.ctypes.data, 0
        else:
            torch = _torch()
            sc = out if out is not None else torch.empty(max(self.nnz, 1), dtype=torch.int32,
                                                         device="cuda")
            ptr, on_dev = sc.data_ptr(), 1
        st = (ctypes.c_uint64 * 3)()
        _check(library().lmgp_fire_scores(self._h, seed, level, int(bool(weighted)),
                                          ctypes.byref(params) if params is not None else None,
                                          _stream_ptr(stream), ptr, on_dev, st))
        return sc[:self.nnz], dict(fires=int(st[0]), burns=int(st[1]), steps=int(st[2]))

    def coarsen(self, k: int, seed: int = 1, params: Optional[Params] = None, stream=None):
        h = ctypes.c_void_p()
        _check(library().lmgp_coarsen(self._h, k, seed,
                                      ctypes.byref(params) if params is not None else None,
                                      _stream_ptr(stream), ctypes.byref(h)))
        return Hierarchy(h, self)


class Hierarchy:
    def __init__(self, handle, graph):
        self._h = handle
        self._graph = graph  # keeps the graph alive

    def close(self):
        if self._h and self._h.value:
            library().lmgp_hierarchy_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    @property
    def levels(self) -> int:
        n = ctypes.c_uint32()
        _check(library().lmgp_hierarchy_levels(self._h, ctypes.byref(n)))
        return int(n.value)

    def info(self, level: int) -> dict:
        li = LevelInfo()
        _check(library().lmgp_hierarchy_level_info(self._h, level, ctypes.byref(li)))
        return li.as_dict()

    def copy_level(self, level: int) -> dict:
        inf = self.info(level)
        n, nnz = inf["n"], 2 * inf["m"]
        xadj = np.empty(n + 1, np.uint64)
        adj = np.empty(nnz, np.uint32)
        vw = np.empty(n, np.int64)
        ew = np.empty(nnz, np.int64)
        mp = np.empty(n, np.uint32) if level + 1 < self.levels else None
        _check(library().lmgp_hierarchy_copy_level(
            self._h, level, xadj.ctypes.data, adj.ctypes.data, vw.ctypes.data, ew.ctypes.data,
            None if mp is None else mp.ctypes.data))
        return dict(n=n, xadj=xadj, adjncy=adj, vwgt=vw, adjwgt=ew, map=mp)


def create_graph(g, validate: bool = False, stream=None, torch_allocator: bool = False,
                 device: Optional[int] = None) -> DeviceGraph:
    """Create a device graph from an object with n, xadj, adjncy and optional
    vwgt / adjwgt (numpy arrays: host copy; torch cuda tensors: device copy)."""
    xadj = g.xadj
    on_device = hasattr(xadj, "is_cuda") and xadj.is_cuda
    keep = []

    def prep(a, dtype):
        if a is None:
            return None
        if on_device:
            return a.contiguous()
        arr = np.ascontiguousarray(a, dtype=dtype) if dtype else np.ascontiguousarray(a)
        keep.append(arr)
        return arr

    xa = prep(xadj, np.uint64)
    adj = prep(g.adjncy, np.uint32)
    vw = prep(getattr(g, "vwgt", None), None)
    ew = prep(getattr(g, "adjwgt", None), None)
    if vw is not None and not on_device and vw.dtype not in (np.int32, np.int64):
        vw = np.ascontiguousarray(vw, np.int64)
        keep.append(vw)
    if ew is not None and not on_device and ew.dtype not in (np.int32, np.int64):
        ew = np.ascontiguousarray(ew, np.int64)
        keep.append(ew)
    n = int(g.n)
    nnz = int(adj.shape[0])
    vp, vb = _ptr(vw)
    ep, eb = _ptr(ew)
    view = CsrView(n, nnz, _ptr(xa)[0], _ptr(adj)[0] if nnz else None, vp, ep, vb, eb,
                   1 if on_device else 0, 1 if validate else 0)
    alloc = None
    if torch_allocator:
        torch = _torch()
        alloc = _TorchAllocator(device if device is not None else torch.cuda.current_device())
    h = ctypes.c_void_p()
    _check(library().lmgp_graph_create(ctypes.byref(view),
                                       ctypes.byref(alloc.struct) if alloc else None,
                                       _stream_ptr(stream), ctypes.byref(h)))
    return DeviceGraph(h.value, n, nnz, keep=None, allocator=alloc)


def partition_batch(graphs: Sequence[DeviceGraph], ks: Sequence[int], epss: Sequence[float],
                    seeds: Sequence[int], params: Optional[Params] = None, stream=None,
                    outs=None):
    """One batched run over several graphs; returns (list of blocks, list of results)."""
    torch = _torch()
    B = len(graphs)
    if outs is None:
        outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
    hs = (ctypes.c_void_p * B)(*[g.handle.value for g in graphs])
    kk = (ctypes.c_uint32 * B)(*ks)
    ee = (ctypes.c_double * B)(*epss)
    ss = (ctypes.c_uint64 * B)(*seeds)
    oo = (ctypes.c_void_p * B)(*[o.data_ptr() for o in outs])
    rr = (Result * B)()
    _check(library().lmgp_partition_batch(hs, kk, ee, ss, B,
                                          ctypes.byref(params) if params is not None else None,
                                          _stream_ptr(stream), oo, 1, rr))
    return outs, [r.as_dict() for r in rr]


class Server:
    """Serving loop: submit partition requests, poll or wait for results."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, max_batch: int = 32,
                 streams: int = 4, ip_device: int = 2, join_runs: bool = False):
        cfg = ServerConfig(hbm_budget_bytes, max_slots, max_batch, streams, ip_device,
                           1 if join_runs else 0)
        h = ctypes.c_void_p()
        _check(library().lmgp_server_create(ctypes.byref(cfg), None, ctypes.byref(h)))
        self._h = h
        self._pending = {}

    def submit(self, graph: DeviceGraph, k: int, eps: float = 0.03, seed: int = 1,
               params: Optional[Params] = None) -> int:
        out = np.empty(graph.n, np.uint32)
        t = ctypes.c_uint64()
        if params is None:
            _check(library().lmgp_server_submit(self._h, graph.handle, k, eps, seed,
                                                out.ctypes.data, ctypes.byref(t)))
        else:
            _check(library().lmgp_server_submit_params(self._h, graph.handle, k, eps, seed,
                                                       ctypes.byref(params), out.ctypes.data,
                                                       ctypes.byref(t)))
        self._pending[int(t.value)] = (out, graph)
        return int(t.value)

    def stats(self) -> dict:
        st = ServerStats()
        _check(library().lmgp_server_stats_read(self._h, ctypes.byref(st)))
        return st.as_dict()

    def poll(self, ticket: int):
        r = Result()
        st = library().lmgp_server_poll(self._h, ticket, ctypes.byref(r))
        if st == 4:  # LMGP_ENOTREADY
            return None
        _check(st)
        out, _ = self._pending.pop(ticket)
        return out, r.as_dict()

    def wait(self, ticket: int):
        r = Result()
        _check(library().lmgp_server_wait(self._h, ticket, ctypes.byref(r)))
        out, _ = self._pending.pop(ticket)
        return out, r.as_dict()

    def close(self):
        if self._h and self._h.value:
            library().lmgp_server_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
