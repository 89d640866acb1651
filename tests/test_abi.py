"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects malformed arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2504_17615_amd as L
from paper_2504_17615_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmgp.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmgp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("lmgp_graph_create", "lmgp_coarsen", "lmgp_partition", "lmgp_partition_batch",
                 "lmgp_server_create", "lmgp_server_submit", "lmgp_server_poll",
                 "lmgp_server_wait", "lmgp_hierarchy_copy_level", "lmgp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert sorted(B.EXPORTED) == declared()


def test_default_params_match_the_paper():
    p = L.default_params()
    assert (p.tau_e_num, p.tau_e_den, p.tau_d_num, p.tau_d_den) == (1, 2, 1, 2)
    assert (p.rho_num, p.rho_den) == (4, 1)
    assert p.clim == 160 and (p.shrink_num, p.shrink_den) == (5, 2)
    assert (p.lp_rounds, p.ref_rounds, p.subrounds, p.max_levels) == (5, 5, 4, 64)


def _view(n, xadj, adj, nnz=None):
    xa = np.ascontiguousarray(xadj, np.uint64)
    ad = np.ascontiguousarray(adj, np.uint32)
    v = B.CsrView(n, len(ad) if nnz is None else nnz, xa.ctypes.data,
                  ad.ctypes.data if len(ad) else None, None, None, 0, 0, 0, 0)
    return v, (xa, ad)


@pytest.mark.parametrize("case", ["empty", "odd_nnz", "null_xadj", "bad_bits", "huge_n"])
def test_graph_create_rejects_malformed_views_on_the_host(case):
    lib = L.library()
    v, keep = _view(3, [0, 1, 2, 2], [1, 0])
    if case == "empty":
        v.n = 0
    elif case == "odd_nnz":
        v.nnz = 3
    elif case == "null_xadj":
        v.xadj = None
    elif case == "bad_bits":
        w = np.ones(2, np.int32)
        keep = keep + (w,)
        v.adjwgt = w.ctypes.data
        v.adjwgt_bits = 16
    elif case == "huge_n":
        v.n = 1 << 31
    h = ctypes.c_void_p()
    st = lib.lmgp_graph_create(ctypes.byref(v), None, None, ctypes.byref(h))
    assert st == 1  # LMGP_EINVAL
    assert lib.lmgp_last_error()
    assert h.value is None


def test_null_arguments_are_rejected():
    lib = L.library()
    assert lib.lmgp_graph_create(None, None, None, None) == 1
    assert lib.lmgp_coarsen(None, 4, 1, None, None, None) == 1
    assert lib.lmgp_partition(None, 4, 0.03, 1, None, None, None, 0, None) == 1
    assert lib.lmgp_hierarchy_levels(None, None) == 1
    assert lib.lmgp_server_create(None, None, None) == 1
    cfg = B.ServerConfig(0, 1, 1, 1, 0)  # zero budget
    h = ctypes.c_void_p()
    assert lib.lmgp_server_create(ctypes.byref(cfg), None, ctypes.byref(h)) == 1


def test_profile_api_without_device():
    L.profile_enable(False)
    assert isinstance(L.profile_read(reset=True), dict)


def test_tuner_api_without_device():
    p = L.default_params()
    assert p.tune == 0  # fixed default class table unless asked
    assert p.ip_device == 2 and p.graph_rounds == 0  # automatic initial partitioning
    L.tuner_clear()
    assert L.tuner_info() == {"entries": 0, "trials": 0}
