"""GPU: device memory of the library's own pool.

Graphs created without a caller allocator work from one caching pool per
device, so that the working memory one call leaves cached serves the next call
on any graph: partitioning many resident graphs one after another must not
keep a working set per graph.
"""
import pytest

from paper_2504_17615_amd import graphgen as gg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_17615_amd as L

    L.library()
    return L


def _used():
    torch.cuda.synchronize()
    free, total = torch.cuda.mem_get_info()
    return total - free


def test_calls_on_many_graphs_share_cached_memory(lib):
    count = 24
    print(f"memory: {count} graphs er(2^17, 2^20)", flush=True)
    dgs = [lib.create_graph(gg.er(1 << 17, 1 << 20, seed=100 + i)) for i in range(count)]
    u0 = _used()
    dgs[0].partition(8, 0.03, 1, host_out=True)
    u1 = _used()
    for i in range(1, count):
        dgs[i].partition(8, 0.03, 1 + i, host_out=True)
    u2 = _used()
    first, rest = u1 - u0, u2 - u1
    print(f"memory: first call {first >> 20} MiB, the {count - 1} others {rest >> 20} MiB", flush=True)
    # one pool per graph would keep about `first` per graph, (count - 1) * first in all
    assert rest <= 4 * max(first, 32 << 20)
