"""Write tests/golden/c4_grad256.json using the oracle only.

Workload (synth.workloads.c4_inputs): 50 taxa x 1500 sites GTR+G4 (seed 4),
256 topologies from a breadth-first NNI walk around the generating tree,
each with its own lengths ~ Exp(mean 0.05).  For every topology the file
stores the oracle's FP64 lnL and its derivative with respect to each of the
97 branch lengths (each edge's derivative from partials recomputed with the
tree re-rooted on that edge).  Values are rounded to 15 significant digits.
Run from the repository root: python tests/golden/make_c4.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import workloads  # noqa: E402
from oracle import core as oc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_grad256.json")

_W = None


def _init():
    global _W
    aln, tops, lens = workloads.c4_inputs()
    _W = (oc.Data.from_alignment(aln), tops, lens)


def _job(i):
    D, tops, lens = _W
    l, g, _ = oc.gradient(D, tops[i], lens[i])
    return i, l, [float("%.15g" % x) for x in g]


def main():
    oc.build(force=False)
    aln, tops, lens = workloads.c4_inputs()
    t0 = time.time()
    res = [None] * len(tops)
    with Pool(min(8, os.cpu_count() or 1), initializer=_init) as pool:
        for r in pool.imap_unordered(_job, range(len(tops))):
            res[r[0]] = r
    out = {
        "workload": "256 NNI-walk topologies, 50 taxa x 1500 sites GTR+G4 (seed 4), lengths ~ Exp(0.05)",
        "n_patterns": int(aln.n_patterns), "tips_sum": int(aln.tips.astype(np.int64).sum()),
        "lens_sum": float(np.sum(lens)),
        "lnl": [r[1] for r in res],
        "grad": [r[2] for r in res],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", OUT, "in %.0fs" % (time.time() - t0))


if __name__ == "__main__":
    main()
