"""Threshold search over NNI neighbourhoods with batched GPU optimisation.

The search follows the topographer's loop (Methods, "Phylogenetic
Topographer"): a FIFO todo queue of candidate topologies, a visited table of
every topology whose branch lengths were fully optimised, and a good table
of those whose optimised lnL is at least lmax + T (T < 0).  Visiting a
topology optimises all its lengths; a good topology proposes each of its
unvisited NNI neighbours, whose lengths are partially optimised and which
join the queue when that partial lnL is at least lmax + T.  Every judgement
of a topology as good uses its fully optimised lnL.  A proposal's partial
optimisation covers the lengths within its radius r of the new edge
(pt_radius_masks: r = 0 the new edge only, r = 1 adds two neighbouring
edges, and so on; r = -1 all edges).

Batching: the queue is consumed a batch at a time, so one batch of visits
and one batch of proposals are each a single persistent launch of the
library's optimiser.  lmax is updated after each batch, and the good table
is filtered by the final lmax + T at the end, so the result does not depend
on the batch size beyond what the paper's own order dependence allows.

Topology identity is the library's canonical split key (sorted non-trivial
splits as bitmasks), hashed on the host in Python sets and dicts.

Starting lengths of a proposal are its parent's lengths carried through the
move (cold start).  With a warm start, a proposal that the cold start's
partial optimum leaves below the gate by at most warm_margin is optimised
again from the parent's lengths with the five edges the move touches
replaced by the network's prediction, and queued if that partial optimum
passes the gate: the good set is then a superset of the cold search's.  A
queued proposal carries its partially optimised lengths to its visit.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L


@dataclass
class SearchResult:
    lmax: float
    good: dict  # key bytes -> (lnL, edges, brlen)
    visited: int
    proposed: int
    queued: int
    full_passes: int
    full_time_s: float
    proposal_time_s: float
    batches: int
    warm_tried: int = 0   # cold-rejected proposals within warm_margin of the gate, retried warm
    warm_passed: int = 0  # of those, the ones whose warm-started partial optimum passed the gate
    samples: list = field(default_factory=list)  # (features, parent lengths, optimised lengths) of the
                                                 # five touched edges, when collecting


class WarmStart:
    """A trained network that predicts the five touched lengths of a move as
    t = (t_parent + shift) * exp(y) - shift."""

    def __init__(self, ctx, params, n_hidden=128, shift=1e-4):
        self.net = L.MLP(ctx, L.PT_NNI_FEATURES, n_hidden, 5, params)
        self.shift = float(shift)

    @classmethod
    def load(cls, ctx, path):
        import json
        d = json.load(open(path))
        return cls(ctx, np.asarray(d["params"], np.float32), d["n_hidden"], d.get("shift", 1e-4))

    def apply(self, d_x, d_pos, d_base, d_brlen, t_min=1e-8, t_max=100.0, stream=None):
        self.net.warm_start(d_x, d_pos, d_base, d_brlen, t_min, t_max, self.shift, stream=stream)


class ThresholdSearch:
    def __init__(self, ctx, aln, threshold=-10.0, radius=0, warm: WarmStart | None = None,
                 precision=L.PT_FP32, batch=1024, opt=None, warm_margin=20.0):
        if threshold >= 0:
            raise ValueError("the threshold offset T must be negative")
        if int(radius) != radius or radius < -1:
            raise ValueError("radius must be an integer >= 0, or -1 for all edges")
        self.ctx, self.aln, self.T, self.radius, self.warm = ctx, aln, float(threshold), int(radius), warm
        self.precision, self.batch = precision, int(batch)
        self.warm_margin = float(warm_margin)
        self.opt = opt if opt is not None else L.opt_default(precision)
        self.n = aln.n_taxa

    def key(self, edges):
        return L.pt_topology_key(self.n, edges).tobytes()

    def _optimize(self, edge_lists, brlen, masks=None, warm_rows=None):
        """Optimises a batch; brlen is the concatenation of the trees' start
        lengths.  warm_rows = (features, pos, base) applies the warm start on
        the device first.  Returns (lnl, brlen, passes)."""
        import torch
        dev = torch.device("cuda", 0)
        T = L.Trees(edge_lists)
        mask = None if masks is None else np.concatenate(masks).astype(np.uint8)
        plan = L.Plan(self.ctx, [self.aln], T, L.PT_PLAN_OPTIMIZE, self.precision, mask=mask)
        stream = torch.cuda.current_stream(dev)
        b = torch.tensor(brlen, dtype=torch.float64, device=dev)
        if warm_rows is not None:
            X, pos, base = warm_rows
            self.warm.apply(torch.tensor(X, device=dev), torch.tensor(pos, device=dev),
                            torch.tensor(base, device=dev), b, self.opt.t_min, self.opt.t_max, stream=stream)
        nt = T.n_trees
        lnl = torch.zeros(nt, dtype=torch.float64, device=dev)
        ps = torch.zeros(nt, dtype=torch.int32, device=dev)
        plan.optimize(b, lnl, ps, None, opt=self.opt, stream=stream)
        torch.cuda.synchronize(dev)
        out = lnl.cpu().numpy(), b.cpu().numpy(), ps.cpu().numpy()
        plan.close()
        return out

    def _propose(self, chunk, radius, stats, warm=False):
        """Partial optimisation of one chunk of proposals, from the parent's
        lengths (cold) or from the network's lengths for the five touched
        edges (warm); returns (lnL per proposal, lengths concatenated)."""
        n = self.n
        E = 2 * n - 3
        trees = [p[1] for p in chunk]
        starts = np.concatenate([p[2] for p in chunk])
        masks = None
        if radius == "touched":
            # the five edges the move touches, the rest held at the parent's
            masks = []
            for p in chunk:
                m = np.zeros(E, np.uint8)
                m[p[4]] = 1
                masks.append(m)
        elif radius >= 0:
            masks = list(L.pt_radius_masks(n, np.stack(trees), [p[4][0] for p in chunk], radius))
        t0 = time.perf_counter()
        rows = None
        if warm:
            X = np.stack([p[3] for p in chunk]).astype(np.float32)
            pos = np.stack([i * E + p[4] for i, p in enumerate(chunk)]).astype(np.int32)
            base = np.stack([p[5][p[4]] for p in chunk])
            rows = (X, pos, base)
        lnl, bo, _ = self._optimize(trees, starts, masks, rows)
        stats["prop_time"] += time.perf_counter() - t0
        return lnl, bo

    def run(self, starts, collect=None, max_samples=None, progress=None):
        """starts: list of (edges, brlen).  With collect = "full", every
        proposal is fully optimised, with collect = "touched" its five
        touched edges are optimised with the rest held at the parent's
        lengths, and (features, parent and optimised lengths of the five
        touched edges) are recorded for training; the proposal's gate uses
        that optimum.  progress, if given, is called with a one-line summary
        after every batch of visits."""
        if collect not in (None, "full", "touched"):
            raise ValueError("collect must be None, 'full' or 'touched'")
        n = self.n
        E = 2 * n - 3
        todo = []  # (key, edges, brlen)
        queued = set()
        for e, b in starts:
            k = self.key(e)
            if k not in queued:
                queued.add(k)
                todo.append((k, np.asarray(e, np.int32), np.asarray(b, np.float64)))
        visited = set()
        good = {}
        lmax = -np.inf
        stats = dict(proposed=0, queued=len(todo), full_passes=0, full_time=0.0, prop_time=0.0, batches=0,
                     warm_tried=0, warm_passed=0)
        samples = []
        n_samples = 0
        head = 0
        while head < len(todo):
            # ---- visit a batch: full optimisation
            batch = []
            while head < len(todo) and len(batch) < self.batch:
                k, e, b = todo[head]
                head += 1
                if k in visited:
                    continue
                visited.add(k)
                batch.append((k, e, b))
            if not batch:
                break
            t0 = time.perf_counter()
            lnl, bo, ps = self._optimize([e for _, e, _ in batch], np.concatenate([b for _, _, b in batch]))
            stats["full_time"] += time.perf_counter() - t0
            stats["full_passes"] += int(ps.sum())
            stats["batches"] += 1
            lmax = max(lmax, float(lnl.max()))
            parents = []
            for i, (k, e, _) in enumerate(batch):
                if lnl[i] >= lmax + self.T:
                    bi = bo[i * E:(i + 1) * E].copy()
                    good[k] = (float(lnl[i]), e, bi)
                    parents.append((e, bi))
            # ---- propose the unvisited neighbours of the good ones.  A key
            # joins the queue only when one of its proposals passes the gate,
            # so a neighbour rejected from one parent's lengths is proposed
            # again by a later good parent (the paper proposes every
            # unvisited neighbour); a key proposed by several parents in one
            # round is optimised once per parent and keeps the best.
            props = []  # (key, edges, start brlen, features row, touched, parent brlen)
            for e, b in parents:
                ne, nb, tt = L.pt_nni_neighbors(n, e, b)
                F = L.pt_nni_features(n, e, b) if (self.warm is not None or collect) else None
                ks = L.pt_topology_keys(n, ne)
                for j in range(len(ne)):
                    k = ks[j].tobytes()
                    if k in visited or k in queued:
                        continue
                    props.append((k, ne[j], nb[j], None if F is None else F[j], tt[j], b))
            stats["proposed"] += len(props)
            if progress is not None:
                progress("batch %d: %d visited, %d good, %d new proposals, lmax %.4f" % (
                    stats["batches"], len(visited), len(good), len(props), lmax))
            radius = {None: self.radius, "full": -1, "touched": "touched"}[collect]
            gate = lmax + self.T
            best = {}  # key -> (partial lnL, edges, lengths)
            near = []  # cold-rejected proposals within warm_margin of the gate
            for s0 in range(0, len(props), self.batch):
                if max_samples is not None and n_samples >= max_samples:
                    break
                chunk = props[s0:s0 + self.batch]
                lnl, bo = self._propose(chunk, radius, stats)
                for i, p in enumerate(chunk):
                    bi = bo[i * E:(i + 1) * E]
                    if collect:
                        tt = p[4]
                        samples.append((p[3], p[5][tt].copy(), bi[tt].copy()))
                        n_samples += 1
                    if lnl[i] >= gate:
                        if p[0] not in best or lnl[i] > best[p[0]][0]:
                            best[p[0]] = (lnl[i], p[1], bi.copy())
                    elif self.warm is not None and lnl[i] >= gate - self.warm_margin:
                        near.append(p)
            # the warm start retries the near misses of the round (one launch
            # per batch of them); a key joins the queue if either start's
            # partial optimum passes the gate, so the gate is never stricter
            # than the cold start's
            near = [p for p in near if p[0] not in best]
            stats["warm_tried"] += len(near)
            for s0 in range(0, len(near), self.batch):
                chunk = near[s0:s0 + self.batch]
                lnl, bo = self._propose(chunk, radius, stats, warm=True)
                for i, p in enumerate(chunk):
                    if lnl[i] >= gate and (p[0] not in best or lnl[i] > best[p[0]][0]):
                        if p[0] not in best:
                            stats["warm_passed"] += 1
                        best[p[0]] = (lnl[i], p[1], bo[i * E:(i + 1) * E].copy())
            for k, (_, e, bi) in best.items():
                queued.add(k)
                todo.append((k, e, bi))
                stats["queued"] += 1
            if max_samples is not None and n_samples >= max_samples:
                break
        final = {k: v for k, v in good.items() if v[0] >= lmax + self.T}
        return SearchResult(lmax=lmax, good=final, visited=len(visited), proposed=stats["proposed"],
                            queued=stats["queued"], full_passes=stats["full_passes"],
                            full_time_s=stats["full_time"], proposal_time_s=stats["prop_time"],
                            batches=stats["batches"], warm_tried=stats["warm_tried"],
                            warm_passed=stats["warm_passed"], samples=samples)


def hls_summary(n, result):
    """Split frequencies and majority-rule consensus of a search's good set
    (Results, "Split Frequency Comparison": topologies weighted by their
    normalised maximised likelihoods).  Returns (splits uint64[m][W],
    frequencies, consensus Newick)."""
    good = list(result.good.values())
    keys = L.pt_topology_keys(n, np.stack([g[1] for g in good]))
    splits, freq = L.pt_split_frequencies(n, keys, np.array([g[0] for g in good]))
    return splits, freq, L.pt_majority_consensus(n, splits, freq)


def main():
    """Threshold searches at several proposal radii on one synthetic workload,
    one JSON line per radius: good, visited and proposed counts, time, and
    the good topologies that the radius -1 search found and this one missed.

      python -m paper_1811_11007_amd.search --seed 6 --radii -1 0 1 2
    """
    import argparse
    import json
    import sys

    from .train_warmstart import optimise_start, workload

    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=6)
    ap.add_argument("--threshold", type=float, default=-10.0)
    ap.add_argument("--radii", type=int, nargs="+", default=[-1, 0, 1, 2])
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--warm", default=None, help="warm-start network weights (JSON)")
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = L.Context(0)
    e, b, aln = workload(args.seed)
    A = L.Alignment.from_synth(ctx, aln)
    b0, l0 = optimise_start(ctx, A, e, b)
    log("seed %d: %d taxa, %d patterns, start lnL %.4f" % (args.seed, aln.n_taxa, aln.n_patterns, l0))
    warm = WarmStart.load(ctx, args.warm) if args.warm else None
    full = None
    for r in args.radii:
        t0 = time.perf_counter()
        res = ThresholdSearch(ctx, A, threshold=args.threshold, radius=r, warm=warm, batch=args.batch).run(
            [(e, b0)], progress=log)
        secs = time.perf_counter() - t0
        good = set(res.good)
        if r == -1 and full is None:
            full = good
        print(json.dumps({
            "seed": args.seed, "radius": r, "threshold": args.threshold, "warm": bool(warm),
            "good": len(good), "visited": res.visited, "proposed": res.proposed, "lmax": round(res.lmax, 4),
            "seconds": round(secs, 2), "proposal_seconds": round(res.proposal_time_s, 2),
            "missed": None if full is None else len(full - good),
            "extra": None if full is None else len(good - full),
            "consensus": hls_summary(aln.n_taxa, res)[2]}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
