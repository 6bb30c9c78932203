"""Write tests/golden/c2_hillclimb.json using the oracle only.

Workload: 27 taxa x 1949 sites simulated under GTR+G4 (exchangeabilities
Dirichlet(1 x 6), frequencies Dirichlet(10 x 4), alpha 0.5) on a Yule tree
with Exp(mean 0.05) branch lengths, generator seed 2.  Starting from the
generating topology, NNI hill-climbing with full FP64 oracle branch
optimisation (best improving neighbour, lengths inherited) reaches a local
maximum; the file stores that tree, its optimised lengths and lnL, and the
oracle's optimised lnL of each of its 2(n-3) = 48 NNI neighbours, keyed by
topology.  Run from the repository root: python tests/golden/make_c2.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import core as oc  # noqa: E402
from oracle import topo  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_hillclimb.json")
N, SITES, SEED = 27, 1949, 2


def c2_data():
    rng = np.random.default_rng(SEED)
    edges, brlen = synth.yule_tree(N, rng, mean=0.05)
    aln = synth.make_alignment(edges, brlen, N, SITES, rng, alpha=0.5, n_cats=4)
    return edges, brlen, aln


_D = None


def _init():
    global _D
    _, _, aln = c2_data()
    _D = oc.Data.from_alignment(aln)


def _opt(args):
    e, b = args
    l, bo, ps, cv = oc.optimize(_D, e, b)
    return l, bo.tolist(), ps, cv


def main():
    oc.build(force=False)
    edges, brlen, aln = c2_data()
    t0 = time.time()
    with Pool(min(8, os.cpu_count() or 1), initializer=_init) as pool:
        cur_e = edges
        cur_l, cur_b, _, _ = pool.map(_opt, [(edges, brlen)])[0]
        cur_b = np.asarray(cur_b)
        steps = 0
        while True:
            nb = topo.nni_neighbors(cur_e, cur_b, N)
            res = pool.map(_opt, nb)
            best = int(np.argmax([r[0] for r in res]))
            print("step %d lnL %.6f best neighbour %.6f (%.0fs)" % (steps, cur_l, res[best][0], time.time() - t0),
                  flush=True)
            if res[best][0] <= cur_l + 1e-6:
                break
            cur_e, cur_l, cur_b = nb[best][0], res[best][0], np.asarray(res[best][1])
            steps += 1
    out = {
        "workload": "27 taxa x 1949 sites GTR+G4, Yule tree, Exp(0.05) lengths, seed 2",
        "n_taxa": N, "n_sites": SITES, "seed": SEED,
        "n_patterns": int(aln.n_patterns), "tips_sum": int(aln.tips.astype(np.int64).sum()),
        "hill_climb_steps": steps,
        "base_edges": np.asarray(cur_e).tolist(), "base_brlen": cur_b.tolist(), "base_lnl": cur_l,
        "oracle": {"t_min": oc.T_MIN, "t_max": oc.T_MAX, "tol_lnl": oc.TOL_LNL, "tol_t": oc.TOL_T},
        "neighbours": [
            {"key": [str(s) for s in topo.key(e, N)], "edges": np.asarray(e).tolist(),
             "start_brlen": np.asarray(b).tolist(), "lnl": r[0], "brlen": r[1], "passes": r[2],
             "converged": bool(r[3])}
            for (e, b), r in zip(nb, res)
        ],
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, "in %.0fs" % (time.time() - t0))


if __name__ == "__main__":
    main()
