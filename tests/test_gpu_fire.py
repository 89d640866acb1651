"""GPU parity of the (Weighted) Forest Fire scores and of the samplers that
threshold on them (Sec. 4.2; the appendix's WFF algorithm) against the
oracle: the scores element by element with the fire and burn counts, and the
hierarchy and partition built with samplers 4 and 5 bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_2504_17615_amd import graphgen as gg
from tests import graphs as T
from tests.test_gpu_parity import check_hierarchy, check_partition

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_17615_amd as L

    L.library()
    return L


def _star(leaves, rng):
    # a hub row longer than the register-held rows (several 64-entry chunks)
    w = rng.integers(1, 9, size=leaves)
    return T.from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)], w)


def _with_isolated(g_base, extra):
    # the graph (unit node weights) plus `extra` isolated nodes at the end
    n = g_base.n + extra
    xadj = np.concatenate([g_base.xadj, np.full(extra, g_base.xadj[-1], g_base.xadj.dtype)])
    return T.G(n=n, xadj=xadj, adjncy=g_base.adjncy, adjwgt=g_base.adjwgt)


def _graph(name):
    rng = np.random.default_rng(7)
    if name == "star1000":  # hub row in the register-mask range (256 < deg <= 4096)
        return _star(1000, rng)
    if name == "star5000":  # hub row beyond it (flags in device memory)
        return _star(5000, rng)
    if name == "rgg14":
        return gg.rgg(1 << 14, seed=3)
    if name == "er12_iso":
        return _with_isolated(gg.er(1 << 12, 1 << 14, seed=2), 500)
    if name == "grid64":
        return gg.grid(64, 64)
    if name == "rmat13":
        return gg.rmat(13, seed=4)
    raise KeyError(name)


CASES = [
    ("rgg14", True, (3, 5), (1, 2)),
    ("rgg14", False, (3, 5), (1, 2)),
    ("rmat13", True, (3, 5), (1, 2)),
    ("rmat13", False, (1, 3), (1, 1)),
    ("er12_iso", True, (1, 1), (3, 2)),
    ("grid64", False, (0, 1), (1, 4)),
    ("star1000", True, (1, 5), (2, 1)),
    ("star1000", False, (0, 1), (5, 1)),
    ("star5000", True, (1, 10), (1, 1)),
    ("star5000", False, (0, 1), (2, 1)),
]


@pytest.mark.parametrize("name,weighted,p,nu", CASES)
def test_fire_scores_match_oracle(lib, name, weighted, p, nu):
    g = _graph(name)
    for seed, level in ((1, 2), (9, 5)):
        print(f"fire {name} n={g.n} nnz={g.nnz} weighted={weighted} p={p} nu={nu} "
              f"seed={seed} level={level}", flush=True)
        dg = lib.create_graph(g, validate=True)
        prm = lib.default_params(ff_p_num=p[0], ff_p_den=p[1], ff_nu_num=nu[0], ff_nu_den=nu[1])
        got, st = dg.fire_scores(seed, level, weighted, prm, host_out=True)
        want, ost = O.fire_scores(g, seed, level, weighted, p, nu)
        assert st["fires"] == ost["fires"] and st["burns"] == ost["burns"], (st, ost)
        assert np.array_equal(got.astype(np.int64), want)
        # device output: the same bits
        dsc, _ = dg.fire_scores(seed, level, weighted, prm)
        torch.cuda.synchronize()
        assert np.array_equal(dsc.cpu().numpy().view(np.uint32).astype(np.int64), want)


def test_fire_scores_edgeless_graph(lib):
    g = T.from_edges(5, np.zeros((0, 2), np.int64))
    dg = lib.create_graph(g)
    got, st = dg.fire_scores(3, 2, True, host_out=True)
    assert st == dict(fires=0, burns=0, steps=0) and got.size == 0


def test_fire_scores_need_sorted_rows(lib):
    g = gg.grid(8, 8)
    perm = g.adjncy.copy()
    for u in range(g.n):  # reverse each row
        a, b = int(g.xadj[u]), int(g.xadj[u + 1])
        perm[a:b] = perm[a:b][::-1]
    dg = lib.create_graph(T.G(n=g.n, xadj=g.xadj, adjncy=perm, adjwgt=g.adjwgt))
    with pytest.raises(lib.LmgpError) as ei:
        dg.fire_scores(1, 2, True, host_out=True)
    assert ei.value.status == 1 and "sorted" in str(ei.value)


@pytest.mark.parametrize("sampler", [4, 5])
@pytest.mark.parametrize("name,k", [("er_1e14", 16), ("rmat13", 16)])
def test_fire_sampler_hierarchy_matches_oracle(lib, sampler, name, k):
    g = gg.er(1 << 14, 1 << 18, seed=5) if name == "er_1e14" else gg.rmat(13, seed=4)
    oh = O.coarsen(g, k, 1, O.params(sampler=sampler))
    if name == "er_1e14":
        assert any(i["triggered"] for i in oh.info[1:])
    check_hierarchy(lib, g, k, 1, sampler=sampler)
    check_partition(lib, g, k, 0.03, 1, sampler=sampler)


def test_fire_sampler_non_default_parameters(lib):
    g = gg.er(1 << 13, 1 << 17, seed=6)
    kw = dict(sampler=5, ff_p_num=1, ff_p_den=4, ff_nu_num=3, ff_nu_den=2)
    check_hierarchy(lib, g, 8, 3, **kw)
