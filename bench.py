"""Benchmark: batched branch-length optimisation of NNI neighbour topologies.

Workload (one step): full branch-length optimisation of all 48 NNI
neighbours of a hill-climbed 27-taxon tree over 1949 sites (976 patterns)
simulated under GTR+G4, lengths inherited from the parent, FP32 partials
with per-pattern scaling and FP64 arithmetic and sums; one persistent
kernel launch replayed from a HIP graph.  A step counts only if every
topology's lnL is within 1e-4 of the FP64 CPU oracle's optimum (stored in
tests/golden/c2_hillclimb.json by a script that calls only the oracle).

Prints one JSON line.  Extra fields: the same batch in FP64, the plain
per-topology GPU path (one tree per call, no graph), the 512-topology batch
over four uneven alignments (optimised in one launch, and its pruning pass),
the all-edge gradient of 256 50-taxon trees, the roofline of the dominant
kernel and the oracle timed on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_hillclimb.json")
GOLDEN3 = os.path.join(ROOT, "tests", "golden", "c3_batch512.json")
GOLDEN4 = os.path.join(ROOT, "tests", "golden", "c4_grad256.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_counters.json")
FP64_VALU_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of the sources that decide the optimiser's work per launch (its
    kernels and the host code that sets its programs and tolerances)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "abi.cpp", "tree.cpp"):
        with open(os.path.join(ROOT, "paper_1811_11007_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def c2_inputs():
    import synth
    g = json.load(open(GOLDEN))
    rng = np.random.default_rng(g["seed"])
    edges, brlen = synth.yule_tree(g["n_taxa"], rng, mean=0.05)
    aln = synth.make_alignment(edges, brlen, g["n_taxa"], g["n_sites"], rng, alpha=0.5, n_cats=4)
    assert aln.n_patterns == g["n_patterns"] and int(aln.tips.astype(np.int64).sum()) == g["tips_sum"], \
        "generator output differs from the stored workload"
    return g, aln


def key_int(k, n):
    W = (n + 63) // 64
    return tuple(sum(int(row[w]) << (64 * w) for w in range(W)) for row in k)


def c3_inputs():
    """Four uneven alignments (27x1949, 36x1812, 50x1133, 64x1008), 128 NNI
    walk topologies each around the generating tree: 512 topologies."""
    from synth import workloads
    return workloads.c3_inputs()


def c4_inputs():
    """256 NNI-walk topologies of a 50-taxon x 1500-site GTR+G4 alignment with
    Exp(mean 0.05) lengths (the gradient workload)."""
    from synth import workloads
    return workloads.c4_inputs()


def c3_golden():
    """Oracle lnL of the 512 topologies at their starting lengths, and the
    local maxima the oracle reaches from three starts (the inherited lengths
    first; tests/golden/c3_batch512.json, written by an oracle-only
    script)."""
    g = json.load(open(GOLDEN3))
    return np.asarray(g["start_lnl"]), np.asarray(g["opt_lnl"]), g["local_optima"]


def stationary_gain(ctx, alns, trees, brlen):
    """Largest predicted gain of one Newton step on any edge of each tree,
    from the FP64 gradient and hessian diagonal at `brlen` (0 on an edge at a
    length bound whose derivative points out of the range)."""
    import paper_1811_11007_amd as pt
    _, g, h = pt.pt_batch_branch_grad(ctx, alns, trees, brlen, pt.PT_FP64, hess=True)
    opt = pt.opt_default(pt.PT_FP64)
    at_lo = (brlen <= opt.t_min * (1 + 1e-9)) & (g <= 0)
    at_hi = (brlen >= opt.t_max * (1 - 1e-9)) & (g >= 0)
    pred = np.where(h < 0, g * g / (2 * np.maximum(-h, 1e-300)), np.inf)
    pred[at_lo | at_hi] = 0.0
    off = trees.edge_offset
    return np.array([pred[off[i]:off[i + 1]].max() for i in range(trees.n_trees)])


def loglik_reg_flops(alns, trees, idx):
    """Algorithmic FP64 flops of the register-resident lnL: per pattern and
    category, each of the n-2 partial updates is two 4x4 matrix-vector
    products and a product of the results (2*32 + 4 = 68 flops), and the root
    edge one matrix-vector product and a weighted dot product (32 + 8)."""
    f = 0.0
    for t, i in zip(trees, idx):
        a = alns[i]
        n = a.n_taxa
        f += a.n_patterns * a.n_cats * ((n - 2) * 68.0 + 40.0)
    return f


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the headline measurement")
    ap.add_argument("--no-search", action="store_true", help="skip the threshold-search extra (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run an elementwise copy of 256 MiB (y = -x, float32) whose known traffic "
                         "calibrates hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the batch runs on a single MI355X "
              "(topologies shard across GPUs with no collective). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1811_11007_amd as pt

    if args.copy_probe:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.neg(x)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (x.numel() * 4, y.numel() * 4))
        del x, y

    g, aln = c2_inputs()
    n = g["n_taxa"]
    base_e = np.asarray(g["base_edges"], np.int32)
    base_b = np.asarray(g["base_brlen"])
    want = {tuple(int(x) for x in nb["key"]): nb["lnl"] for nb in g["neighbours"]}

    ctx = pt.Context(0)
    A = pt.Alignment.from_synth(ctx, aln)
    ne, nbl, _ = pt.pt_nni_neighbors(n, base_e, base_b)
    keys = [key_int(pt.pt_topology_key(n, e), n) for e in ne]
    assert set(keys) == set(want), "NNI neighbours differ from the stored workload"
    ref = np.array([want[k] for k in keys])
    T = pt.Trees(list(ne))
    NT = T.n_trees
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()

    def run_batch(precision, steps, warmup, graphs=True, tune=True):
        plan = pt.Plan(ctx, [A], T, pt.PT_PLAN_OPTIMIZE, precision)
        b0 = torch.tensor(nbl.ravel(), dtype=torch.float64, device=dev)
        b = torch.empty_like(b0)
        lnl = torch.zeros(NT, dtype=torch.float64, device=dev)
        ps = torch.zeros(NT, dtype=torch.int32, device=dev)
        st = torch.zeros(NT, dtype=torch.int32, device=dev)
        shape = None
        with torch.cuda.stream(stream):
            if tune:
                plan.autotune(b0)
                shape = plan.launch_shape()
            plan.set_graphs(graphs)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]

            def step(i=None):
                b.copy_(b0, non_blocking=True)
                if i is not None:
                    ev[i][0].record(stream)
                plan.optimize(b, lnl, ps, st, stream=stream)
                if i is not None:
                    ev[i][1].record(stream)

            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                step(i)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        kern_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
        passes = ps.cpu().numpy()
        res = dict(ms=(t1 - t0) * 1e3 / steps, kern_ms=kern_ms, lnl=lnl.cpu().numpy(), passes=passes,
                   status=st.cpu().numpy(), bytes=plan.traffic(pt.PT_PLAN_OPTIMIZE, passes), shape=shape)
        plan.close()
        return res

    log("fp32 batch ...")
    r32 = run_batch(pt.PT_FP32, args.steps, args.warmup)
    d32 = np.abs(r32["lnl"] - ref)
    ok = bool(np.all(d32 <= 1e-4))
    value = NT / (r32["ms"] / 1e3)
    achieved = r32["bytes"] / (r32["kern_ms"] / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC):
        tr = json.load(open(TRAFFIC))
        if tr.get("kernel_hash") == kernel_hash():
            # the counters of the launch shape this run's autotuner chose
            shape = "%dx%d" % (r32["shape"][0], r32["shape"][2])
            traffic = tr.get("optimize_c2_fp32", {}).get(shape, {}).get("bytes_per_launch")
    out = {
        "metric": "optimized topologies/s at |dlnL|<1e-4; pruning HBM GB/s vs peak",
        "value": round(value if ok else 0.0, 3),
        "unit": "topologies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 partials and partial updates / f64 Newton sums and lnL",
        "data": "synthetic (seeded GTR+G4 simulation; no dataset)",
        "config": {"workload": "48 NNI neighbours of a hill-climbed 27-taxon tree, 1949 sites "
                               "(%d patterns) GTR+G4, full branch optimisation" % aln.n_patterns,
                   "topologies_per_step": NT, "precision": "fp32 partials + per-pattern scaling",
                   "launch": {"block": r32["shape"][0], "items_per_thread": r32["shape"][1],
                              "blocks_per_tree": r32["shape"][2], "hip_graph": True}},
        "parity": {"max_abs_dlnl_vs_oracle": float(d32.max()), "all_within_1e-4": ok,
                   "status_converged": int(np.sum(r32["status"] == 0)),
                   "passes_mean": float(r32["passes"].mean())},
        "roofline": {"bound": "hbm", "kernel": "k_optimize",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": r32["bytes"], "kernel_ms": round(r32["kern_ms"], 4)},
    }
    if not args.no_extras:
        log("fp64 batch ...")
        r64 = run_batch(pt.PT_FP64, max(3, args.steps // 4), 1)
        out["fp64"] = {"value": round(NT / (r64["ms"] / 1e3), 3), "ms_per_step": round(r64["ms"], 4),
                       "max_rel_dlnl_vs_oracle": float(np.max(np.abs(r64["lnl"] - ref) / np.abs(ref))),
                       "max_abs_dlnl_vs_oracle": float(np.max(np.abs(r64["lnl"] - ref)))}
        log("per-topology path ...")
        # plain per-topology GPU path: same kernel, one tree per plan and call, no graph
        plans = [pt.Plan(ctx, [A], pt.Trees([ne[i]]), pt.PT_PLAN_OPTIMIZE, pt.PT_FP32) for i in range(NT)]
        bs = [torch.tensor(nbl[i], dtype=torch.float64, device=dev) for i in range(NT)]
        ls = [torch.zeros(1, dtype=torch.float64, device=dev) for _ in range(NT)]
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(NT):
                bs[i].copy_(torch.tensor(nbl[i], dtype=torch.float64))
                plans[i].optimize(bs[i], ls[i], stream=stream)
                stream.synchronize()
            t1 = time.perf_counter()
        pl_l = np.array([float(x.item()) for x in ls])
        out["per_topology_path"] = {"value": round(NT / (t1 - t0), 3), "unit": "topologies/s",
                                    "max_abs_dlnl_vs_oracle": float(np.max(np.abs(pl_l - ref)))}
        out["batched_over_per_topology"] = round(value / out["per_topology_path"]["value"], 2)
        for p_ in plans:
            p_.close()

        log("gamma-shape optimisation ...")
        # per-topology model optimisation: lengths and Gamma shape jointly, the
        # same 48 neighbours, FP32 partials, starting at the alignment's alpha
        plan_a = pt.Plan(ctx, [A], T, pt.PT_PLAN_OPTIMIZE | pt.PT_PLAN_LOGLIK, pt.PT_FP32)
        ba = torch.tensor(nbl.ravel(), dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            plan_a.set_graphs(True)
            plan_a.optimize_alpha(ba, np.full(NT, aln.alpha), stream=stream)  # graphs captured
            ba.copy_(torch.tensor(nbl.ravel(), dtype=torch.float64))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            la, aa, ra = plan_a.optimize_alpha(ba, np.full(NT, aln.alpha), stream=stream)
            t1 = time.perf_counter()
        out["gamma_shape"] = {"workload": "the same 48 neighbours, branch lengths and Gamma shape alpha jointly "
                                          "(rounds of batched length optimisation and lockstep Brent on log "
                                          "alpha), FP32 partials",
                              "value": round(NT / (t1 - t0), 3), "unit": "topologies/s",
                              "rounds": int(ra), "alpha_range": [round(float(aa.min()), 4),
                                                                 round(float(aa.max()), 4)],
                              "mean_lnl_gain_over_fixed_alpha": round(float(np.mean(la - r32["lnl"])), 4)}
        plan_a.close()

        log("pruning on 512 topologies ...")
        alns3, trees3, lens3, idx3 = c3_inputs()
        start3, same3, opt3 = c3_golden()
        A3 = [pt.Alignment.from_synth(ctx, a) for a in alns3]
        T3 = pt.Trees(trees3, idx3)
        b3 = torch.tensor(lens3, dtype=torch.float64, device=dev)
        reps = 20

        tiles3 = {}

        def time_loglik(precision, path):
            plan = pt.Plan(ctx, A3, T3, pt.PT_PLAN_LOGLIK, precision)
            plan.set_loglik_path(path)
            if path == pt.PT_LOGLIK_STORED:
                tiles3[precision] = plan.autotune_tiles(b3)
            l = torch.zeros(T3.n_trees, dtype=torch.float64, device=dev)
            with torch.cuda.stream(stream):
                plan.set_graphs(True)
                for _ in range(3):
                    plan.loglik(b3, l, stream=stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    plan.loglik(b3, l, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            by = plan.traffic(pt.PT_PLAN_LOGLIK)
            plan.close()
            return ms, by, l.cpu().numpy()

        # the stored post-order pass (every partial written to and read from
        # HBM, as in an optimisation's first pass or a gradient's lower half)
        ms3, by3, l3 = time_loglik(pt.PT_FP32, pt.PT_LOGLIK_STORED)
        ms3d, by3d, l3d = time_loglik(pt.PT_FP64, pt.PT_LOGLIK_STORED)
        # the register-resident pass (no partial stored)
        ms3r, by3r, l3r = time_loglik(pt.PT_FP32, pt.PT_LOGLIK_REGISTERS)
        flops3r = loglik_reg_flops(alns3, trees3, idx3)
        d3 = float(np.max(np.abs(l3d - l3)))
        # batching: all 512 topologies optimised in one persistent launch
        plan3o = pt.Plan(ctx, A3, T3, pt.PT_PLAN_OPTIMIZE, pt.PT_FP32)
        bo0 = torch.tensor(lens3, dtype=torch.float64, device=dev)
        bo = torch.empty_like(bo0)
        lo = torch.zeros(T3.n_trees, dtype=torch.float64, device=dev)
        po = torch.zeros(T3.n_trees, dtype=torch.int32, device=dev)
        with torch.cuda.stream(stream):
            plan3o.autotune(bo0)
            shape3 = plan3o.launch_shape()
            plan3o.set_graphs(True)
            bo.copy_(bo0, non_blocking=True)
            plan3o.optimize(bo, lo, po, stream=stream)
            torch.cuda.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            for _ in range(3):
                bo.copy_(bo0, non_blocking=True)
                plan3o.optimize(bo, lo, po, stream=stream)
            f1.record(stream)
            torch.cuda.synchronize()
        ms3o = f0.elapsed_time(f1) / 3
        by3o = plan3o.traffic(pt.PT_PLAN_OPTIMIZE, po.cpu().numpy())
        lo_h = lo.cpu().numpy()
        # distance to the nearest of the oracle's stored local maxima of each
        # topology; an optimum elsewhere (the ascent's path picks the maximum)
        # must be stationary by the FP64 gradient kernel and above its start
        d3o = np.array([min(abs(lo_h[i] - x) for x in opt3[i]) for i in range(len(opt3))])
        other3 = np.nonzero(d3o > 1e-4)[0]
        gain3 = stationary_gain(ctx, A3, T3, bo.cpu().numpy())
        ok3o = bool(len(other3) <= 16 and np.all(gain3[other3] < 1e-3) and np.all(lo_h[other3] > start3[other3]))
        out["batched_512"] = {"workload": "512 NNI-walk topologies over 27x1949, 36x1812, 50x1133, 64x1008 "
                                          "GTR+G4, full optimisation, FP32 partials, one persistent launch",
                              "value": round(T3.n_trees / (ms3o / 1e3) if ok3o else 0.0, 2), "unit": "topologies/s",
                              "ms_per_batch": round(ms3o, 3), "launch": list(shape3),
                              "passes_mean": float(po.float().mean()), "passes_max": int(po.max().item()),
                              "at_stored_oracle_maximum": int(len(opt3) - len(other3)),
                              "elsewhere": {str(int(i)): {"dlnl_vs_same_start_oracle": round(float(lo_h[i] - same3[i]), 4),
                                                          "predicted_gain": float(gain3[i])} for i in other3},
                              "max_abs_dlnl_at_stored_maximum": float(np.delete(d3o, other3).max()),
                              "gate_ok": ok3o,
                              "at_same_start_oracle_optimum": int(np.sum(np.abs(lo_h - same3) <= 1e-4)),
                              "achieved_GBs": round(by3o / (ms3o / 1e3) / 1e9, 1)}
        plan3o.close()
        log("gradient of 256 trees ...")
        aln4, tops4, lens4 = c4_inputs()
        A4 = pt.Alignment.from_synth(ctx, aln4)
        T4 = pt.Trees(tops4)
        plan4 = pt.Plan(ctx, [A4], T4, pt.PT_PLAN_GRAD, pt.PT_FP32)
        b4 = torch.tensor(lens4.ravel(), dtype=torch.float64, device=dev)
        l4 = torch.zeros(T4.n_trees, dtype=torch.float64, device=dev)
        g4 = torch.zeros_like(b4)
        tiles4 = plan4.autotune_tiles(b4)
        with torch.cuda.stream(stream):
            plan4.set_graphs(True)
            for _ in range(3):
                plan4.grad(b4, l4, g4, stream=stream)
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(stream)
            for _ in range(10):
                plan4.grad(b4, l4, g4, stream=stream)
            g1.record(stream)
            torch.cuda.synchronize()
        ms4 = g0.elapsed_time(g1) / 10
        by4 = plan4.traffic(pt.PT_PLAN_GRAD)
        out["gradient"] = {"workload": "all 97 branch-length gradients of 256 topologies, 50 taxa x 1500 sites "
                                       "GTR+G4, FP32 partials (adjoint: lower and upper partials, one edge "
                                       "derivative per edge)",
                           "ms_per_call": round(ms4, 4), "trees_per_s": round(T4.n_trees / (ms4 / 1e3), 1),
                           "algorithmic_bytes": by4, "achieved_GBs": round(by4 / (ms4 / 1e3) / 1e9, 1),
                           "frac_of_peak": round(by4 / (ms4 / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                           "patterns_per_tile": tiles4}
        # the stored oracle gradients of the same trees (tests/golden/c4_grad256.json)
        g4_want = np.asarray(json.load(open(GOLDEN4))["grad"]).ravel()
        e4 = float(np.max(np.abs(g4.cpu().numpy() - g4_want) / np.maximum(1.0, np.abs(g4_want))))
        out["gradient"]["max_err_vs_oracle"] = e4
        out["gradient"]["all_within_1e-3"] = e4 < 1e-3
        plan4.close()
        out["pruning"] = {"workload": "512 topologies over 27x1949, 36x1812, 50x1133, 64x1008 GTR+G4, FP32 "
                                      "partials stored in HBM (the post-order pass that starts an optimisation "
                                      "or a gradient)",
                          "ms_per_call": round(ms3, 4), "algorithmic_bytes": by3,
                          "achieved_GBs": round(by3 / (ms3 / 1e3) / 1e9, 1),
                          "frac_of_peak": round(by3 / (ms3 / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "counter_GBs": None,
                          "max_abs_dlnl_vs_oracle": float(np.max(np.abs(l3 - start3))),
                          "all_within_1e-4": bool(np.max(np.abs(l3 - start3)) <= 1e-4),
                          "note": "graph of k_pmat + k_tiles + k_reduce",
                          "patterns_per_tile": tiles3.get(pt.PT_FP32),
                          "fp64": {"ms_per_call": round(ms3d, 4), "algorithmic_bytes": by3d,
                                   "achieved_GBs": round(by3d / (ms3d / 1e3) / 1e9, 1),
                                   "frac_of_peak": round(by3d / (ms3d / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                   "max_rel_dlnl_vs_oracle": float(np.max(np.abs(l3d - start3) / np.abs(start3))),
                                   "patterns_per_tile": tiles3.get(pt.PT_FP64),
                                   "max_abs_dlnl_vs_fp32": d3}}
        d3r = np.abs(l3r - start3)
        out["loglik_registers"] = {
            "workload": "lnL of the same 512 topologies with no partial stored (FP64 partials of each "
                        "pattern and category in registers and an LDS stack)",
            "ms_per_call": round(ms3r, 4), "trees_per_s": round(T3.n_trees / (ms3r / 1e3), 1),
            "speedup_over_stored_fp32": round(ms3 / ms3r, 2),
            "max_abs_dlnl_vs_oracle": float(d3r.max()), "all_within_1e-4": bool(np.all(d3r <= 1e-4)),
            "roofline": {"bound": "alu", "achieved": round(flops3r / (ms3r / 1e3) / 1e12, 3),
                         "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flops3r / (ms3r / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4),
                         "flops_per_call": flops3r, "bytes_per_call": by3r},
            "note": "graph of k_pmat + k_loglik_reg + k_reduce"}
        if not args.no_search:
            log("threshold search, cold and warm-started ...")
            # the learned warm start in the threshold search (T = -10, radius-0
            # proposals, batch 1024, FP32 partials) on the network's held-out
            # 64-taxon x 2500-site alignment (seed 6): the cold start gates every
            # proposal, the network's lengths retry the near misses
            from paper_1811_11007_amd import search as S
            from paper_1811_11007_amd.train_warmstart import optimise_start, workload
            e5, b5, aln5 = workload(6)
            A5 = pt.Alignment.from_synth(ctx, aln5)
            b5o, _ = optimise_start(ctx, A5, e5, b5)
            warm = S.WarmStart.load(ctx, os.path.join(ROOT, "paper_1811_11007_amd", "warmstart_64x2500.json"))
            runs = {}
            for name, w in (("cold", None), ("warm", warm), ("cold_again", None)):
                t0 = time.perf_counter()
                res = S.ThresholdSearch(ctx, A5, threshold=-10.0, radius=0, warm=w, batch=1024).run([(e5, b5o)])
                runs[name] = (time.perf_counter() - t0, res)
            rc, rw = runs["cold_again"][1], runs["warm"][1]
            out["search"] = {
                "workload": "threshold search T=-10, radius-0 proposals, batch 1024, FP32 partials, held-out "
                            "64 taxa x 2500 sites (seed 6), from the optimised generating tree",
                "cold": {"seconds": round(runs["cold_again"][0], 3), "good": len(rc.good), "visited": rc.visited,
                         "proposed": rc.proposed, "full_passes": rc.full_passes,
                         "proposal_seconds": round(rc.proposal_time_s, 3), "visit_seconds": round(rc.full_time_s, 3)},
                "warm": {"seconds": round(runs["warm"][0], 3), "good": len(rw.good), "visited": rw.visited,
                         "proposed": rw.proposed, "full_passes": rw.full_passes,
                         "proposal_seconds": round(rw.proposal_time_s, 3), "visit_seconds": round(rw.full_time_s, 3),
                         "near_misses_retried": rw.warm_tried, "retries_passed": rw.warm_passed},
                "warm_contains_cold": set(rc.good) <= set(rw.good),
                "good_only_warm": len(set(rw.good) - set(rc.good)),
                "good_only_cold": len(set(rc.good) - set(rw.good)),
                "warm_over_cold_time": round(runs["warm"][0] / runs["cold_again"][0], 3),
                "note": "the first cold run warms up plan memory and is not reported"}
        log("copy bandwidth ...")
        xc = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        yc = torch.empty_like(xc)
        xc.fill_(1.0)
        with torch.cuda.stream(stream):
            for _ in range(3):
                yc.copy_(xc)
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            for _ in range(10):
                yc.copy_(xc)
            c1.record(stream)
            torch.cuda.synchronize()
        msc = c0.elapsed_time(c1) / 10
        out["copy_bandwidth"] = {"workload": "device-to-device copy of 1 GiB (torch copy_), read + write bytes",
                                 "GBs": round(2 * xc.numel() * 4 / (msc / 1e3) / 1e9, 1),
                                 "frac_of_peak": round(2 * xc.numel() * 4 / (msc / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del xc, yc
        if os.path.exists(TRAFFIC):
            tr = json.load(open(TRAFFIC))
            if tr.get("kernel_hash") == kernel_hash():
                # measured FETCH_SIZE + WRITE_SIZE bytes per launch of each
                # path's main kernel (scaled by the copy probe's counts), over
                # the whole call's time (a lower bound for the kernel alone)
                def counter(key, ms):
                    return round(tr[key]["bytes_per_launch"] / (ms / 1e3) / 1e9, 1) if key in tr else None
                # (the tile kernels' counters at the tile size this run chose)
                out["pruning"]["counter_GBs"] = counter("tiles_512_fp32_t%d" % tiles3[pt.PT_FP32], ms3)
                out["pruning"]["fp64"]["counter_GBs"] = counter("tiles_512_fp64_t%d" % tiles3[pt.PT_FP64], ms3d)
                out["loglik_registers"]["roofline"]["traffic"] = tr.get("loglik_reg_512", {}).get("bytes_per_launch")
                out["batched_512"]["counter_GBs"] = counter("optimize_512_fp32", ms3o)
                out["gradient"]["counter_GBs"] = counter("grad_256_fp32_t%d" % tiles4, ms4)

    if not args.no_cpu:
        log("oracle cpu baseline ...")
        from concurrent.futures import ThreadPoolExecutor
        from oracle import core as oc
        D = oc.Data.from_alignment(aln)
        # one thread: the first neighbours for about 10 s
        t0 = time.perf_counter()
        done = 0
        while done < len(ne) and (time.perf_counter() - t0) < 10.0:
            oc.optimize(D, ne[done], nbl[done])
            done += 1
        dt1 = time.perf_counter() - t0
        # every host thread of this process's share (the C oracle releases the
        # interpreter lock and keeps no global state): all 48 neighbours
        threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda i: oc.optimize(D, ne[i], nbl[i]), range(len(ne))))
        dtn = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(ne) / dtn, 4), "unit": "topologies/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "all 48 neighbours, FP64 oracle full optimisation (its own tolerances), "
                                         "%d threads, %.1f s" % (threads, dtn),
                               "single_thread": {"value": round(done / dt1, 4),
                                                 "sample": "first %d neighbours, %.1f s" % (done, dt1)},
                               "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
