"""Write tests/golden/c3_batch512.json using the oracle only.

Workload (synth.workloads.c3_inputs): four GTR+G4 alignments of 27x1949,
36x1812, 50x1133 and 64x1008 taxa x sites (seeds 31-34), 128 topologies
each from a breadth-first NNI walk around the generating tree, lengths
inherited from it.  For every one of the 512 topologies the file stores the
oracle's FP64 lnL at the starting lengths and its fully optimised lnL
(coordinate-wise safeguarded Newton to its own tolerances), with the passes
it took.

The lnL surface over branch lengths can have several local maxima, and
which one an ascent reaches depends on its path (edge order, step rule).
So the oracle also optimises every topology from two further starts that
do not depend on any other code: every length 0.05, and the inherited
lengths each multiplied by a factor drawn uniformly from [0.5, 2] (numpy
generator seeded with 1000 + the topology's index).  The distinct optima
found (within 1e-6 relative) are stored as the topology's known local
maxima; an optimiser started from the inherited lengths is expected to
reach one of them.  Run from the repository root:
python tests/golden/make_c3.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_batch512.json")

_W = None


def _init():
    global _W
    alns, trees, lens, idx = workloads.c3_inputs()
    offs = np.concatenate([[0], np.cumsum([len(t) for t in trees])])
    _W = ([oc.Data.from_alignment(a) for a in alns], trees, lens, idx, offs)


def _job(i):
    D, trees, lens, idx, offs = _W
    d = D[idx[i]]
    b = lens[offs[i]:offs[i + 1]]
    start = oc.loglik(d, trees[i], b)
    l, _, ps, cv = oc.optimize(d, trees[i], b)
    rng = np.random.default_rng(1000 + i)
    optima = [l]
    for b2 in (np.full(len(b), 0.05), b * rng.uniform(0.5, 2.0, size=len(b))):
        l2, _, _, cv2 = oc.optimize(d, trees[i], b2)
        if cv2 and all(abs(l2 - x) > 1e-6 * abs(x) for x in optima):
            optima.append(l2)
    return i, start, l, ps, cv, sorted(optima, reverse=True)


def main():
    oc.build(force=False)
    alns, trees, lens, idx = workloads.c3_inputs()
    t0 = time.time()
    res = [None] * len(trees)
    # longest jobs (the largest trees) first
    order = sorted(range(len(trees)), key=lambda i: -int(idx[i]))
    with Pool(min(int(os.environ.get("MAKE_WORKERS", "8")), os.cpu_count() or 1), initializer=_init) as pool:
        for k, r in enumerate(pool.imap_unordered(_job, order)):
            res[r[0]] = r
            if (k + 1) % 32 == 0:
                print("%d / %d (%.0fs)" % (k + 1, len(trees), time.time() - t0), flush=True)
    out = {
        "workload": "512 NNI-walk topologies over 27x1949, 36x1812, 50x1133, 64x1008 GTR+G4 (seeds 31-34), "
                    "lengths inherited from the generating tree",
        "alignments": [{"n_taxa": int(a.n_taxa), "n_patterns": int(a.n_patterns),
                        "tips_sum": int(a.tips.astype(np.int64).sum())} for a in alns],
        "edges_sum": int(sum(int(np.asarray(t, np.int64).sum()) for t in trees)),
        "lens_sum": float(np.sum(lens)),
        "oracle": {"t_min": oc.T_MIN, "t_max": oc.T_MAX, "tol_lnl": oc.TOL_LNL, "tol_t": oc.TOL_T},
        "start_lnl": [r[1] for r in res],
        "opt_lnl": [r[2] for r in res],
        "passes": [r[3] for r in res],
        "converged": [bool(r[4]) for r in res],
        "local_optima": [r[5] for r in res],
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, "in %.0fs" % (time.time() - t0))


if __name__ == "__main__":
    main()
