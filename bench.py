#!/usr/bin/env python3
"""Benchmark: SCC labels of synthetic digraphs on one MI355X.

Default workload: the batched configuration, 4096 independent digraphs
(vertex counts log-uniform in [1e3, 1e6], family uniform among the 2-D torus,
R-MAT edge factor 8 and 3-D k-NN k=5; 590M vertices, 2.9G arcs), resident in
HBM, labelled by scc_labels_batched with the schedule the autotuner picked
on half of the graphs.  One step = one scc_labels_batched call over the whole
batch (trim, first-SCC searches, every multi-source batch, relabels,
canonical labels of every graph).  Beside it, outside the timed region: the
same batch with the default schedule, with the default schedule plus the
learned policy, and as a loop of one plain scc_labels call per graph.

Single-graph workloads (--workload): one step = one scc_labels call.

Prints one JSON line.  ``value`` = input arcs / wall time of a step
(edges/s).  ``roofline`` covers the dominant frontier kernel, from its
algorithmic bytes and its HIP-event time over the timed steps.
``cpu_baseline`` times the Tarjan oracle on the host cores (batched: a thread
pool over the independent graphs).

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload batched4096]
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
                       "family uniform in {torus p=0.5, R-MAT edge factor 8, 3-D k-NN k=5}, run as disjoint "
                       "unions with an autotuned schedule"),
    "sqr_10000": (5, "the paper's SQR lattice: 10000x10000 torus, each endpoint orients each of its edges at "
                     "random, duplicates removed (1.5 arcs per edge)"),
    "rec_1000x10000": (6, "the paper's REC lattice: 1000x10000 torus, each endpoint orients each of its edges at "
                          "random, duplicates removed (1.5 arcs per edge)"),
    "sqr2_10000": (7, "the paper's SQR' lattice: 10000x10000 torus, each arc of each edge kept with p=0.3"),
    "rec2_1000x10000": (8, "the paper's REC' lattice: 1000x10000 torus, each arc of each edge kept with p=0.3"),
}
DEFAULT_WORKLOAD = "batched4096"
BATCH_G, BATCH_LO, BATCH_SEED = 4096, 3.0, 1004
# the frontier kernels timed with options.timing (SCC_KERNEL_* in hipscc.h)
KERNEL_SHORT = ["k_expand0", "k_expand1", "k_pull", "k_heavy0", "k_heavy1", "k_extract", "k_union"]
NK = len(KERNEL_SHORT)


def kernel_name(kind, app="scc", first_slot=1, packed=False):
    """rocprofv3's name of the kernel that timing kind `kind` brackets: the
    expand and edge-parallel kernels are instantiated per search mode (0
    single source, 1 multi-source, 2 multi-source with first-source slots,
    3 LDD of connectivity, 4 LE-lists BFS, 5 first-source slots in packed
    per-vertex records)."""
    single = {"scc": 0, "cc": 3, "le": 0}[app]
    multi = {"scc": (5 if packed else 2) if first_slot else 1, "cc": 1, "le": 4}[app]
    return ["hipscc::k_expand<%d, 1>" % single, "hipscc::k_expand<%d, 1>" % multi, "hipscc::k_pull",
            "hipscc::k_expand_heavy<%d>" % single, "hipscc::k_expand_heavy<%d>" % multi, "hipscc::k_bag_extract",
            "hipscc::k_cc_union"][kind]


def packed_used(opts, st):
    """Whether a call ran its multi-source batches on packed records: the
    library's rule (options.packed = -1: when more than half the vertices
    survive trimming), from the call's statistics."""
    if not opts.first_slot or opts.packed == 0:
        return False
    return opts.packed == 1 or 2 * (st["n"] - st["trimmed"]) > st["n"]


CPU_POOL = 16  # host threads for the multicore oracle (the CPU share of one GPU)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_04934_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel):
    """Counter-measured HBM bytes per launch from profiles/, if taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (KERNEL_SHORT[kernel], workload))
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def host_info():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline_single(g, target_s=20.0, max_runs=5):
    """Tarjan oracle on one core: 1 warm-up, then up to max_runs timed runs
    while their sum stays near target_s (mean and minimum reported)."""
    import oracle
    t0 = time.perf_counter()
    lab = oracle.scc_graph(g)
    warm = time.perf_counter() - t0
    ts = []
    while len(ts) < max_runs and (not ts or sum(ts) + ts[-1] <= target_s):
        t0 = time.perf_counter()
        oracle.scc_graph(g)
        ts.append(time.perf_counter() - t0)
    t = sum(ts) / len(ts)
    info = host_info()
    return lab, {"value": g.m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
                 "sample": "whole graph; sequential Tarjan oracle, 1 warm-up (%.2f s) then %d timed run(s): "
                           "mean %.3f s, min %.3f s" % (warm, len(ts), t, min(ts)),
                 "host": info}


def cpu_baseline_batched(n_of, oo, oa, vb, ab, runs=3):
    """Tarjan oracle over the independent graphs of a batch, a thread pool of
    CPU_POOL host threads (the oracle runs in C and releases the GIL).
    1 warm-up (its labels are the parity reference), then `runs` timed runs."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    G = len(vb) - 1
    threads = max(1, min(CPU_POOL, os.cpu_count() or 1))
    order = sorted(range(G), key=lambda g: -int(ab[g + 1] - ab[g]))  # largest first

    def one(g):
        lo = int(vb[g]) + g
        n = int(vb[g + 1] - vb[g])
        return g, oracle.scc_labels(n, oo[lo:lo + n + 1], oa[int(ab[g]):int(ab[g + 1])])

    def sweep():
        with ThreadPoolExecutor(threads) as ex:
            return dict(ex.map(one, order))

    t0 = time.perf_counter()
    labels = sweep()
    warm = time.perf_counter() - t0
    log("oracle warm-up over %d graphs on %d threads: %.1f s" % (G, threads, warm))
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        sweep()
        ts.append(time.perf_counter() - t0)
    t = sum(ts) / len(ts)
    m = int(ab[-1])
    return labels, {"value": m / t, "unit": "edges/s", "cores": threads, "kind": "oracle",
                    "sample": "every graph of the batch; sequential Tarjan oracle per graph on a pool of %d host "
                              "threads, 1 warm-up (%.1f s) then %d timed runs: mean %.2f s, min %.2f s"
                              % (threads, warm, runs, t, min(ts)),
                    "host": host_info()}


def roofline(ms_k, launches_k, bytes_k, dom, workload, name):
    if launches_k[dom] <= 0 or ms_k[dom] <= 0:
        return None
    per_launch_ms = ms_k[dom] / launches_k[dom]
    per_launch_bytes = bytes_k[dom] / launches_k[dom]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(workload, dom),
            "avg_launch_ms": per_launch_ms, "alg_bytes_per_launch": per_launch_bytes}


def parse_variants(text):
    """'k=v,k=v;k=v' -> list of option-override dicts (A/B runs in one process)."""
    out = []
    for part in filter(None, (p.strip() for p in text.split(";"))):
        d = {}
        for kv in part.split(","):
            k, v = kv.split("=")
            d[k.strip()] = float(v) if "." in v else int(v)
        out.append(d)
    return out


def time_variants(call, base, variants, steps):
    """Whole-call times of option variants (no kernel events): a warm-up
    call, then `steps` timed calls each."""
    import torch

    import paper_2303_04934_amd as scc
    res = []
    for v in variants:
        o = scc.default_options()
        for f, _ in o._fields_:
            setattr(o, f, getattr(base, f))
        o.timing = 0
        for k, x in v.items():
            setattr(o, k, x)
        call(o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call(o)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        log("variant %s: %.3f ms per call" % (v, ms))
        res.append({"options": v, "ms_per_call": ms})
    return res


def load_policy(scc):
    import numpy as np
    scc.policy_load(np.load(os.path.join(ROOT, "paper_2303_04934_amd", "policy_weights.npy")))


def run_batched(args, desc):
    """The batched workload: many graphs resident in HBM, one
    scc_labels_batched call per step with the autotuned schedule."""
    import numpy as np
    import torch

    import graphgen
    import paper_2303_04934_amd as scc
    from paper_2303_04934_amd import autotune

    t0 = time.perf_counter()
    spec = graphgen.batched_spec(BATCH_G, BATCH_SEED, BATCH_LO, args.batch_hi)
    graphs = []
    for i in range(0, BATCH_G, 256):  # generated in slices, with progress lines
        graphs += graphgen.batched_slice(BATCH_G, BATCH_SEED, BATCH_LO, args.batch_hi, i, min(BATCH_G, i + 256))
        log("generated %d/%d graphs (%.0f s)" % (len(graphs), BATCH_G, time.perf_counter() - t0))
    assert len(graphs) == len(spec)
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    del graphs  # the oracle reads per-graph views of the concatenated arrays
    log("generated %d graphs, n=%d m=%d in %.1f s" % (BATCH_G, vb[-1], ab[-1], time.perf_counter() - t0))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to("cuda:0")
    arrs = (dev(oo), dev(oa), dev(io), dev(ia))
    del io, ia
    load_policy(scc)
    base = scc.default_options(validate=0)
    t0 = time.perf_counter()
    if args.schedule:
        # a given schedule (profiling runs repeat the one the timed run picked)
        opts = scc.default_options(validate=0)
        tau, beta, beta_fast, policy = args.schedule.split(",")
        opts.tau, opts.beta, opts.beta_fast, opts.policy = int(tau), float(beta), float(beta_fast), int(policy)
        opts.graph_rounds = args.graph_rounds
        tuned = {"given": args.schedule}
    else:
        opts, tuned = autotune.tune(vb, ab, *arrs, base_options=base)
    log("autotune picked tau=%d beta=%.1f beta_fast=%.0f policy=%d in %.1f s (held out: %.1f ms tuned vs %.1f "
        "default)" % (opts.tau, opts.beta, opts.beta_fast, opts.policy, time.perf_counter() - t0,
                      tuned.get("held_out_tuned_ms", 0), tuned.get("held_out_default_ms", 0)))
    # warm-up; its last call times every frontier kernel to pick the dominant one
    for i in range(max(args.warmup, 1)):
        opts.timing = (1 << NK) - 1 if i == max(args.warmup, 1) - 1 else 0
        _, st = scc.scc_labels_batched(vb, ab, *arrs, options=opts, return_stats=True)
    dom = max(range(NK), key=lambda i: st["ms_kernel"][i])
    probe_ms = list(st["ms_kernel"])
    opts.timing = 0 if args.graph_rounds else 1 << dom
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, st = scc.scc_labels_batched(vb, ab, *arrs, options=opts, return_stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    got = out.cpu().numpy()
    log("timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3))
    if args.profile_only:
        rec = {"workload": "batched4096", "ms_per_step": dt * 1e3, "steps": args.steps,
               "schedule": [opts.tau, opts.beta, opts.beta_fast, opts.policy]}
        if args.variants:
            rec["variants"] = time_variants(lambda o: scc.scc_labels_batched(vb, ab, *arrs, options=o), opts,
                                            parse_variants(args.variants), args.steps)
        print(json.dumps(rec), flush=True)
        return

    # comparisons (untimed region), with the same event overhead as the timed steps
    def once(o):
        o.timing = opts.timing
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = scc.scc_labels_batched(vb, ab, *arrs, options=o)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3, r
    default_ms, r_def = once(scc.default_options(validate=0))
    learned_ms, r_lrn = once(scc.default_options(validate=0, policy=1))
    same_def = bool(torch.equal(r_def, out))
    same_lrn = bool(torch.equal(r_lrn, out))
    del r_def, r_lrn
    log("one scc_labels call per graph ...")
    plain = scc.default_options(validate=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_same = True
    for g in range(BATCH_G):
        n, lo = int(vb[g + 1] - vb[g]), int(vb[g]) + g
        dg = scc.DeviceGraph(n, int(ab[g + 1] - ab[g]), arrs[0][lo:lo + n + 1], arrs[1][int(ab[g]):int(ab[g + 1])],
                             arrs[2][lo:lo + n + 1], arrs[3][int(ab[g]):int(ab[g + 1])])
        r = scc.scc_labels(dg, plain)
        loop_same = loop_same and bool(torch.equal(r, out[int(vb[g]):int(vb[g + 1])]))
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    log("default schedule %.1f ms, default + learned policy %.1f ms, per-graph loop %.1f ms"
        % (default_ms, learned_ms, loop_ms))
    m = int(ab[-1])
    line = {
        "metric": METRIC, "value": m / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batched4096", "description": desc, "graphs": BATCH_G, "n": int(vb[-1]), "m": m,
                   "seed": BATCH_SEED, "size_exponents": [BATCH_LO, args.batch_hi], "tau": opts.tau,
                   "beta": opts.beta, "beta_fast": opts.beta_fast, "policy": "learned" if opts.policy == 1 else
                   "fixed", "schedule": "autotuned"},
        "batched_vs_plain": {
            "autotuned_batched_ms": dt * 1e3, "default_batched_ms": default_ms,
            "default_batched_learned_policy_ms": learned_ms, "per_graph_loop_ms": loop_ms,
            "speedup_vs_per_graph_loop": loop_ms / (dt * 1e3), "labels_identical": same_def and same_lrn and loop_same,
            "autotune": tuned},
    }
    ms_k = [sum(s["ms_kernel"][i] for s in stats) for i in range(NK)]
    la_k = [sum(s["launches_kernel"][i] for s in stats) for i in range(NK)]
    by_k = [sum(s["bytes_kernel"][i] for s in stats) for i in range(NK)]
    rf = roofline(ms_k, la_k, by_k, dom, "batched4096",
                  kernel_name(dom, "scc", opts.first_slot, packed_used(opts, stats[-1])))
    if rf:
        rf["launches_per_step"] = la_k[dom] / args.steps
        # the unions run on concurrent streams, so the kernel's summed launch
        # time per step can exceed the step's wall time
        rf["kernel_ms_per_step_summed_over_streams"] = ms_k[dom] / args.steps
        rf["union_streams_option"] = opts.union_streams  # 0: the library picks (two streams)
        line["roofline"] = rf
    last = stats[-1]
    line["stats"] = {"kernel_ms_warmup_call": {KERNEL_SHORT[i]: probe_ms[i] for i in range(NK)},
                     "batches": last["batches"], "rounds_first": last["rounds_first"],
                     "rounds_multi": last["rounds_multi"], "table_restarts": last["table_restarts"],
                     "n_scc": last["n_scc"], "bytes_alg": last["bytes_alg"],
                     "alg_GBps_whole_step": last["bytes_alg"] / dt / 1e9}
    if not args.no_cpu_baseline:
        want, cb = cpu_baseline_batched(None, oo, oa, vb, ab)
        ok = all(np.array_equal(want[g], got[vb[g]:vb[g + 1]]) for g in range(BATCH_G))
        line["cpu_baseline"] = cb
        line["parity"] = "bit-exact vs oracle (every graph)" if ok else "MISMATCH vs oracle"
    print(json.dumps(line), flush=True)
    if line.get("parity", "").startswith("MISMATCH") or not line["batched_vs_plain"]["labels_identical"]:
        sys.exit(1)


def run_single(args, cfg, desc):
    import numpy as np
    import torch

    import graphgen
    import paper_2303_04934_amd as scc

    t0 = time.perf_counter()
    g = graphgen.config(cfg, shrink=args.shrink)
    log("generated %s n=%d m=%d in %.1f s" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    dg = scc.to_device(g, "cuda:0")
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    opts = scc.default_options(timing=0, validate=0, policy=args.policy)
    if args.tau:
        opts.tau = args.tau
    if args.first_slot >= 0:
        opts.first_slot = args.first_slot
    opts.vgc_measure = args.vgc_measure
    opts.graph_rounds = args.graph_rounds
    if args.policy == 1:
        load_policy(scc)
    # Untimed warm-up.  Its last call times every frontier kernel to find the
    # dominant one; the timed steps then bracket only that kernel's launches
    # with events (each event pair costs a little, so the others run bare).
    for i in range(max(args.warmup, 1)):
        opts.timing = (1 << NK) - 1 if i == max(args.warmup, 1) - 1 else 0
        _, st = scc.scc_labels(dg, opts, out=out, return_stats=True)
    dom = max(range(NK), key=lambda i: st["ms_kernel"][i])
    probe_ms = list(st["ms_kernel"])
    # (captured round blocks record no per-kernel events: an A/B run of them
    # times whole calls only)
    opts.timing = 0 if args.graph_rounds else 1 << dom
    torch.cuda.synchronize()
    log("warmup done; dominant frontier kernel %s" % kernel_name(dom, "scc", opts.first_slot))
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = scc.scc_labels(dg, opts, return_stats=True, out=out)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    got = out.cpu().numpy()
    log("timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3))
    line = {
        "metric": METRIC, "value": g.m / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": g.n, "m": g.m, "seed": 1000 + cfg,
                   "tau": opts.tau, "policy": "learned" if args.policy == 1 else "fixed",
                   "first_slot": opts.first_slot, "vgc_measure": opts.vgc_measure,
                   "graph_rounds": opts.graph_rounds, "shrink": args.shrink},
    }
    ms_k = [sum(s["ms_kernel"][i] for s in stats) for i in range(NK)]
    la_k = [sum(s["launches_kernel"][i] for s in stats) for i in range(NK)]
    by_k = [sum(s["bytes_kernel"][i] for s in stats) for i in range(NK)]
    rf = roofline(ms_k, la_k, by_k, dom, args.workload,
                  kernel_name(dom, "scc", opts.first_slot, packed_used(opts, stats[-1])))
    if rf:
        rf["launches_per_step"] = la_k[dom] / args.steps
        rf["kernel_share_of_step"] = ms_k[dom] / args.steps / (dt * 1e3)
        line["roofline"] = rf
    last = stats[-1]
    line["stats"] = {k: last[k] for k in ("ms_trim", "ms_first", "ms_multi", "ms_resize", "ms_label", "batches",
                                         "rounds_first", "rounds_multi", "dense_rounds", "trimmed", "n_scc",
                                         "arcs_scanned", "claims", "claims_table", "bag_inserts", "table_restarts",
                                         "bytes_alg")}
    line["stats"]["alg_GBps_whole_step"] = last["bytes_alg"] / dt / 1e9
    if args.variants:
        line["variants"] = time_variants(lambda o: scc.scc_labels(dg, o, out=out), opts, parse_variants(args.variants),
                                         args.steps)
    # every frontier kernel's event time in the (untimed) warm-up call that picked the dominant one
    line["stats"]["kernel_ms_warmup_call"] = {KERNEL_SHORT[i]: probe_ms[i] for i in range(NK)}
    if not args.no_cpu_baseline:
        want, cb = cpu_baseline_single(g)
        line["cpu_baseline"] = cb
        ok = bool(np.array_equal(got, want))
        line["parity"] = "bit-exact vs oracle" if ok else "MISMATCH vs oracle"
    print(json.dumps(line), flush=True)
    if line.get("parity", "").startswith("MISMATCH"):
        sys.exit(1)


def run_app(args, cfg, desc):
    """Connectivity (Algorithm 4) or LE-lists (Algorithm 5) on the symmetrised
    workload graph: one step = one scc_cc / scc_le_lists call."""
    import numpy as np
    import torch

    import graphgen
    import oracle
    import paper_2303_04934_amd as scc

    t0 = time.perf_counter()
    g = graphgen.symmetrize(graphgen.config(cfg, shrink=args.shrink))
    log("generated %s (symmetrised) n=%d m=%d in %.1f s" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    dg = scc.to_device(g, "cuda:0")
    opts = scc.default_options(validate=0)
    if args.tau:
        opts.tau = args.tau

    def call(o):
        if args.app == "cc":
            return scc.scc_cc(dg, o, return_stats=True)
        return scc.scc_le_lists(dg, o, return_stats=True)
    for i in range(max(args.warmup, 1)):
        opts.timing = (1 << NK) - 1 if i == max(args.warmup, 1) - 1 else 0
        _, st = call(opts)
    dom = max(range(NK), key=lambda i: st["ms_kernel"][i])
    probe_ms = list(st["ms_kernel"])
    opts.timing = 1 << dom
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, st = call(opts)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log("timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3))
    line = {
        "metric": METRIC, "value": g.m / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "%s_%s_sym" % (args.app, args.workload), "app": args.app,
                   "description": "symmetrised " + desc, "n": g.n, "m": g.m, "shrink": args.shrink,
                   "tau": opts.tau, "ldd_beta": opts.ldd_beta, "beta": opts.beta},
    }
    ms_k = [sum(s["ms_kernel"][i] for s in stats) for i in range(NK)]
    la_k = [sum(s["launches_kernel"][i] for s in stats) for i in range(NK)]
    by_k = [sum(s["bytes_kernel"][i] for s in stats) for i in range(NK)]
    rf = roofline(ms_k, la_k, by_k, dom, "%s_%s_sym" % (args.app, args.workload), kernel_name(dom, args.app))
    if rf:
        rf["launches_per_step"] = la_k[dom] / args.steps
        rf["kernel_share_of_step"] = ms_k[dom] / args.steps / (dt * 1e3)
        line["roofline"] = rf
    last = stats[-1]
    line["stats"] = {k: last[k] for k in ("ms_first", "ms_multi", "ms_label", "batches", "rounds_first",
                                         "rounds_multi", "n_scc", "arcs_scanned", "claims", "bag_inserts",
                                         "table_restarts", "bytes_alg")}
    line["stats"]["kernel_ms_warmup_call"] = {KERNEL_SHORT[i]: probe_ms[i] for i in range(NK)}
    if args.variants:
        line["variants"] = time_variants(lambda o: call(o), opts, parse_variants(args.variants), args.steps)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        if args.app == "cc":
            want = oracle.wcc_labels(g.n, g.out_off, g.out_adj)
            ok = bool(np.array_equal(res.cpu().numpy(), want))
        else:
            order, loff, src, dist = (x.cpu().numpy() for x in res)
            wl, ws, wd = oracle.le_lists(g.n, g.out_off, g.out_adj, order)
            ok = bool(np.array_equal(loff, wl) and np.array_equal(src, ws) and np.array_equal(dist, wd))
            line["stats"]["list_entries"] = int(len(ws))
        t = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": g.m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
                                "sample": "whole graph, one run of the sequential oracle (%s), %.2f s"
                                          % ("union-find" if args.app == "cc" else "source-by-source pruned BFS", t),
                                "host": host_info()}
        line["parity"] = "bit-exact vs oracle" if ok else "MISMATCH vs oracle"
    print(json.dumps(line), flush=True)
    if line.get("parity", "").startswith("MISMATCH"):
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--shrink", type=int, default=0, help="reduce n by 2**shrink (exploration only)")
    ap.add_argument("--app", default="scc", choices=["scc", "cc", "le"],
                    help="scc (default), or connectivity / LE-lists on the symmetrised workload graph")
    ap.add_argument("--tau", type=int, default=0, help="VGC budget (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--policy", type=int, default=0, help="0 fixed budget, 1 learned per-round policy")
    ap.add_argument("--first-slot", type=int, default=-1, help="options.first_slot (-1: the library default)")
    ap.add_argument("--vgc-measure", type=int, default=0, help="options.vgc_measure (0 arcs, 1 claims)")
    ap.add_argument("--graph-rounds", type=int, default=0, help="options.graph_rounds (captured round blocks)")
    ap.add_argument("--variants", default="", help="also time option variants: 'k=v,k=v;k=v' (A/B, one process)")
    ap.add_argument("--batch-hi", type=float, default=6.0,
                    help="batched workload: vertex counts log-uniform in [1e3, 10**batch_hi]")
    ap.add_argument("--schedule", default="", help="batched: tau,beta,beta_fast,policy instead of autotuning")
    ap.add_argument("--profile-only", action="store_true",
                    help="batched: only the warm-up and timed steps (for profiler runs)")
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
    if args.app != "scc":
        if args.workload == "batched4096":
            print("--app %s runs on a single-graph workload" % args.app, file=sys.stderr)
            sys.exit(2)
        run_app(args, cfg, desc)
    elif args.workload == "batched4096":
        run_batched(args, desc)
    else:
        run_single(args, cfg, desc)


if __name__ == "__main__":
    main()
