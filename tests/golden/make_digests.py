"""Write tests/golden/digest_<workload>.json from the CPU oracle only.

For the full-size workloads the oracle takes minutes, so its output is stored
as SHA-256 digests of every hierarchy level (CSR, weights, fine-to-coarse map,
level statistics) and of the final block array, plus cut and balance.  The
GPU tests recompute the same digests from the library's output.

usage: python tests/golden/make_digests.py rmat22 er22 rgg24 grid128
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2504_17615_amd import graphgen as gg  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digest(name: str) -> dict:
    g, k, eps, seed = gg.workload(name)
    t0 = time.time()
    h = O.coarsen(g, k, seed)
    levels = []
    for i, lv in enumerate(h.levels):
        levels.append(dict(info=h.info[i], xadj=sha(lv.xadj.astype(np.uint64)),
                           adjncy=sha(lv.adjncy.astype(np.uint32)),
                           vwgt=sha(lv.vwgt.astype(np.int64)),
                           adjwgt=sha(lv.adjwgt.astype(np.int64)),
                           map=sha(h.maps[i].astype(np.uint32)) if i < len(h.maps) else None))
    del h
    t1 = time.time()
    blocks, res, times = O.partition(g, k, eps, seed)
    t2 = time.time()
    return dict(workload=name, n=g.n, m=g.m, k=k, eps=eps, seed=seed, levels=levels,
                blocks=sha(blocks.astype(np.uint32)), result=res,
                oracle_seconds=dict(coarsen_call=round(t1 - t0, 1), partition_call=round(t2 - t1, 1),
                                    phases={p: round(v, 2) for p, v in times.items()}))


if __name__ == "__main__":
    for name in sys.argv[1:]:
        d = digest(name)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"digest_{name}.json")
        with open(out, "w") as f:
            json.dump(d, f, indent=1)
        print(name, d["result"], d["oracle_seconds"], flush=True)
