#!/usr/bin/env python3
"""Benchmark: SCC labels of a synthetic digraph on one MI355X.

One step = one full scc_labels call (trim, first-SCC searches, every
multi-source batch, relabels, canonical labels) on a graph already resident
in HBM.  Prints one JSON line.  ``value`` = input arcs / wall time of a step
(edges/s).  ``roofline`` covers the dominant kernel (the frontier-expansion
kernel of the mode that took longest), from its algorithmic bytes and its
HIP-event time measured over the timed steps.  ``cpu_baseline`` times the
sequential Tarjan oracle on the same graph on one host core.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload rmat_s24_ef16]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SCC wall time + traversed edges/s and HBM GB/s; learned/batched vs plain GPU"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "torus1000_p0.5": (0, "2-D torus 1000x1000, each of the 4 neighbour arcs kept with p=0.5"),
    "rmat_s24_ef16": (1, "R-MAT scale 24, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), self loops and "
                         "duplicates removed, ids randomly permuted"),
    "knn_10M_k5": (2, "directed 5-NN graph of 1e7 points, mixture of 1000 isotropic Gaussians (sigma .01) "
                      "in the unit cube, ties to the lower id"),
    "grid10000_p0.5": (3, "2-D grid 10000x10000 (no wrap), each neighbour arc kept with p=0.5"),
    "batched4096": (4, "4096 graphs, vertex counts log-uniform in [1e3, 10^hi] (hi = --batch-hi, default 6), "
                       "family uniform in {torus p=0.5, R-MAT edge factor 8, 3-D k-NN k=5}, run as one disjoint "
                       "union with an autotuned schedule"),
}
BATCH_G, BATCH_LO, BATCH_SEED = 4096, 3.0, 1004
# the frontier kernels timed with options.timing, as rocprofv3 names them
KERNEL_NAMES = ["hipscc::k_expand<0, 1>", "hipscc::k_expand<1, 1>", "hipscc::k_pull", "hipscc::k_expand_heavy<0>",
                "hipscc::k_expand_heavy<1>", "hipscc::k_bag_extract"]
KERNEL_SHORT = ["k_expand0", "k_expand1", "k_pull", "k_heavy0", "k_heavy1", "k_extract"]
NK = len(KERNEL_NAMES)


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_04934_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, mode):
    """Counter-measured HBM bytes per launch from profiles/, if taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (KERNEL_SHORT[mode], workload))
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(g, runs):
    import oracle
    ts = []
    lab = None
    for _ in range(runs):
        t0 = time.perf_counter()
        lab = oracle.scc_graph(g)
        ts.append(time.perf_counter() - t0)
    t = sum(ts) / len(ts)
    return lab, {"value": g.m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
                 "sample": "whole graph, %d run(s) of the sequential Tarjan oracle, mean %.3f s" % (runs, t)}


def run_batched(args, desc):
    """The batched workload: many graphs resident in HBM, one scc_labels_batched
    call per step with the schedule the autotuner picked; the same batch run
    with the default schedule and as a loop of per-graph scc_labels calls is
    timed once for comparison (outside the timed region)."""
    import numpy as np
    import torch

    import graphgen
    import oracle
    import paper_2303_04934_amd as scc
    from paper_2303_04934_amd import autotune

    t0 = time.perf_counter()
    spec = graphgen.batched_spec(BATCH_G, BATCH_SEED, BATCH_LO, args.batch_hi)
    graphs = []
    for i in range(0, BATCH_G, 256):  # generated in slices, with progress lines
        graphs += graphgen.batched_slice(BATCH_G, BATCH_SEED, BATCH_LO, args.batch_hi, i, min(BATCH_G, i + 256))
        print("[bench] generated %d/%d graphs (%.0f s)" % (len(graphs), BATCH_G, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    assert len(graphs) == len(spec)
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    print("[bench] generated %d graphs, n=%d m=%d in %.1f s" % (len(graphs), vb[-1], ab[-1], time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to("cuda:0")
    arrs = (dev(oo), dev(oa), dev(io), dev(ia))
    base = scc.default_options(validate=0)
    t0 = time.perf_counter()
    opts, tuned = autotune.tune(vb, ab, *arrs, base_options=base)
    print("[bench] autotune picked tau=%d beta=%.1f beta_fast=%.0f in %.1f s" % (opts.tau, opts.beta, opts.beta_fast,
                                                                           time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    # warm-up; its last call times every frontier kernel to pick the dominant one
    for i in range(max(args.warmup, 1)):
        opts.timing = (1 << NK) - 1 if i == max(args.warmup, 1) - 1 else 0
        _, st = scc.scc_labels_batched(vb, ab, *arrs, options=opts, return_stats=True)
    dom = max(range(NK), key=lambda i: st["ms_kernel"][i])
    probe_ms = list(st["ms_kernel"])
    opts.timing = 1 << dom
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, st = scc.scc_labels_batched(vb, ab, *arrs, options=opts, return_stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    got = out.cpu().numpy()
    print("[bench] timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3), file=sys.stderr, flush=True)
    # comparisons (untimed region): default schedule, and one scc_labels call per graph
    base.timing = opts.timing  # the same event overhead as the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scc.scc_labels_batched(vb, ab, *arrs, options=base)
    base.timing = 0
    torch.cuda.synchronize()
    default_ms = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_out = []
    print("[bench] one scc_labels call per graph ...", file=sys.stderr, flush=True)
    for g in range(len(graphs)):
        n, lo = int(vb[g + 1] - vb[g]), int(vb[g]) + g
        dg = scc.DeviceGraph(n, int(ab[g + 1] - ab[g]), arrs[0][lo:lo + n + 1], arrs[1][int(ab[g]):int(ab[g + 1])],
                             arrs[2][lo:lo + n + 1], arrs[3][int(ab[g]):int(ab[g + 1])])
        loop_out.append(scc.scc_labels(dg, base))
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    loop_same = all(np.array_equal(loop_out[g].cpu().numpy(), got[vb[g]:vb[g + 1]]) for g in range(len(graphs)))
    print("[bench] default schedule %.1f ms, per-graph loop %.1f ms" % (default_ms, loop_ms), file=sys.stderr,
          flush=True)
    m = int(ab[-1])
    line = {
        "metric": METRIC, "value": m / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batched4096", "description": desc, "graphs": len(graphs), "n": int(vb[-1]), "m": m,
                   "seed": BATCH_SEED, "size_exponents": [BATCH_LO, args.batch_hi], "tau": opts.tau,
                   "beta": opts.beta, "beta_fast": opts.beta_fast, "schedule": "autotuned"},
        "batched_vs_plain": {"autotuned_batched_ms": dt * 1e3, "default_batched_ms": default_ms,
                             "per_graph_loop_ms": loop_ms, "loop_labels_identical": loop_same,
                             "autotune": tuned},
    }
    per_launch_ms = sum(s["ms_kernel"][dom] for s in stats) / max(1, sum(s["launches_kernel"][dom] for s in stats))
    per_launch_bytes = sum(s["bytes_kernel"][dom] for s in stats) / max(1, sum(s["launches_kernel"][dom] for s in stats))
    if per_launch_ms > 0:
        achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
        line["roofline"] = {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                            "avg_launch_ms": per_launch_ms, "alg_bytes_per_launch": per_launch_bytes}
    line["stats"] = {"kernel_ms_warmup_call": {KERNEL_SHORT[i]: probe_ms[i] for i in range(NK)},
                     "batches": stats[-1]["batches"], "rounds_first": stats[-1]["rounds_first"],
                     "rounds_multi": stats[-1]["rounds_multi"]}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        ok = True
        for g, gr in enumerate(graphs):
            ok = ok and bool(np.array_equal(oracle.scc_graph(gr), got[vb[g]:vb[g + 1]]))
            if g % 512 == 511:
                print("[bench] oracle %d/%d graphs (%.0f s)" % (g + 1, len(graphs), time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        t = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
                                "sample": "every graph of the batch, sequential Tarjan oracle, %.1f s" % t}
        line["parity"] = "bit-exact vs oracle" if ok else "MISMATCH vs oracle"
    print(json.dumps(line), flush=True)
    if line.get("parity", "").startswith("MISMATCH"):
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat_s24_ef16", choices=sorted(WORKLOADS))
    ap.add_argument("--shrink", type=int, default=0, help="reduce n by 2**shrink (exploration only)")
    ap.add_argument("--tau", type=int, default=0, help="VGC budget (0: the library default)")
    ap.add_argument("--cpu-runs", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--policy", type=int, default=0, help="0 fixed budget, 1 learned per-round policy")
    ap.add_argument("--batch-hi", type=float, default=6.0,
                    help="batched workload: vertex counts log-uniform in [1e3, 10**batch_hi]")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    cfg, desc = WORKLOADS[args.workload]
    if args.workload == "batched4096":
        run_batched(args, desc)
        return

    import numpy as np
    import torch

    import graphgen
    import paper_2303_04934_amd as scc

    t0 = time.perf_counter()
    g = graphgen.config(cfg, shrink=args.shrink)
    print("[bench] generated %s n=%d m=%d in %.1f s" % (args.workload, g.n, g.m, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    dg = scc.to_device(g, "cuda:0")
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    opts = scc.default_options(timing=0, validate=0, policy=args.policy)
    if args.tau:
        opts.tau = args.tau
    if args.policy == 1:
        import numpy as np
        scc.policy_load(np.load(os.path.join(ROOT, "paper_2303_04934_amd", "policy_weights.npy")))
    # Untimed warm-up.  Its last call times every frontier kernel to find the
    # dominant one; the timed steps then bracket only that kernel's launches
    # with events (each event pair costs a little, so the others run bare).
    for i in range(max(args.warmup, 1)):
        opts.timing = (1 << NK) - 1 if i == max(args.warmup, 1) - 1 else 0
        _, st = scc.scc_labels(dg, opts, out=out, return_stats=True)
    dom = max(range(NK), key=lambda i: st["ms_kernel"][i])
    probe_ms = list(st["ms_kernel"])
    opts.timing = 1 << dom
    torch.cuda.synchronize()
    print("[bench] warmup done; dominant frontier kernel %s" % KERNEL_NAMES[dom], file=sys.stderr, flush=True)

    ms_exp = [0.0] * NK
    launches = [0] * NK
    bexp = [0] * NK
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = scc.scc_labels(dg, opts, return_stats=True, out=out)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for st in stats:
        for m in range(NK):
            ms_exp[m] += st["ms_kernel"][m]
            launches[m] += st["launches_kernel"][m]
            bexp[m] += st["bytes_kernel"][m]
    got = out.cpu().numpy()
    print("[bench] timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3), file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": g.m / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": g.n, "m": g.m, "seed": 1000 + cfg,
                   "tau": opts.tau, "policy": "learned" if args.policy == 1 else "fixed",
                   "shrink": args.shrink},
    }
    if launches[dom] > 0 and ms_exp[dom] > 0:
        per_launch_ms = ms_exp[dom] / launches[dom]
        per_launch_bytes = bexp[dom] / launches[dom]
        achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
        traffic = load_traffic(args.workload, dom)
        line["roofline"] = {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                            "avg_launch_ms": per_launch_ms, "launches_per_step": launches[dom] / args.steps,
                            "alg_bytes_per_launch": per_launch_bytes,
                            "kernel_share_of_step": ms_exp[dom] / args.steps / (dt * 1e3)}
    last = stats[-1]
    line["stats"] = {k: last[k] for k in ("ms_trim", "ms_first", "ms_multi", "ms_resize", "ms_label", "batches",
                                         "rounds_first", "rounds_multi", "dense_rounds", "trimmed", "n_scc",
                                         "arcs_scanned",
                                         "claims", "bag_inserts", "table_restarts", "bytes_alg")}
    line["stats"]["alg_GBps_whole_step"] = last["bytes_alg"] / dt / 1e9
    # every frontier kernel's event time in the (untimed) warm-up call that picked the dominant one
    line["stats"]["kernel_ms_warmup_call"] = {KERNEL_SHORT[i]: probe_ms[i] for i in range(NK)}
    if not args.no_cpu_baseline:
        want, cb = cpu_baseline(g, args.cpu_runs)
        line["cpu_baseline"] = cb
        ok = bool(np.array_equal(got, want))
        line["parity"] = "bit-exact vs oracle" if ok else "MISMATCH vs oracle"
    print(json.dumps(line), flush=True)
    if line.get("parity", "").startswith("MISMATCH"):
        sys.exit(1)


if __name__ == "__main__":
    main()
