"""Write tests/golden/warm64_heldout.json using the oracle only.

Workload: the held-out alignment of the warm-start network, 64 taxa x 2500
sites simulated under GTR+G4 (exchangeabilities Dirichlet(1 x 6),
frequencies Dirichlet(10 x 4), alpha 0.5) on a Yule tree with Exp(mean
0.05) branch lengths, generator seed 6.  The oracle fully optimises the
generating topology from its simulated lengths, then four of its NNI
neighbours (oracle NNI order) from the lengths they inherit; the file
stores each topology's split key and optimised lnL.  Run from the
repository root: python tests/golden/make_warm64.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warm64_heldout.json")
N, SITES, SEED = 64, 2500, 6
PICK = [0, 17, 61, 121]


def data():
    rng = np.random.default_rng(SEED)
    edges, brlen = synth.yule_tree(N, rng, mean=0.05)
    aln = synth.make_alignment(edges, brlen, N, SITES, rng, alpha=0.5, n_cats=4)
    return edges, brlen, aln


def job(args):
    e, b = args
    _, _, aln = data()
    D = oc.Data.from_alignment(aln)
    lnl, _, passes, conv = oc.optimize(D, e, b)
    assert conv
    return lnl, passes


def main():
    t0 = time.time()
    e, b, aln = data()
    D = oc.Data.from_alignment(aln)
    l0, bo, p0, conv = oc.optimize(D, e, b)
    assert conv
    nbs = topo.nni_neighbors(e, bo, N)
    with Pool(len(PICK)) as pool:
        res = pool.map(job, [nbs[i] for i in PICK])
    out = {"seed": SEED, "n_taxa": N, "n_sites": SITES, "n_patterns": int(aln.n_patterns),
           "start": {"key": [str(k) for k in topo.key(e, N)], "lnl": l0, "passes": p0},
           "neighbours": [{"index": i, "key": [str(k) for k in topo.key(nbs[i][0], N)], "lnl": r[0],
                           "passes": r[1]} for i, r in zip(PICK, res)],
           "seconds": round(time.time() - t0, 1)}
    json.dump(out, open(OUT, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
