"""GPU parity: the HIP path against the sequential oracle, element by element.

SCC labels are integers, so the bar is bit-exact equality with the oracle's
canonical labels (min vertex id per SCC).  Reachability pairs are a set, so the
test sorts both sides and compares exactly.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def check_labels(scc, g, opts=None, name=""):
    say("scc_labels", name or g.name, "n=%d m=%d" % (g.n, g.m))
    dg = scc.to_device(g)
    got, st = scc.scc_labels(dg, opts, return_stats=True)
    got = got.cpu().numpy()
    want = oracle.scc_graph(g)
    assert np.array_equal(got, want), "labels differ on %s (first bad vertex %s)" % (
        name or g.name, np.nonzero(got != want)[0][:5])
    assert st["n_scc"] == len(np.unique(want))
    return st


def as_pairs(p):
    return np.asarray(p).reshape(-1, 2)


def test_tiny_random_graphs(gpu):
    for t in range(60):
        n = 1 + (t * 7) % 150
        g = graphgen.random_digraph(n, [0.7, 1.2, 2.0, 4.0][t % 4], seed=9000 + t, self_loops=(t % 5 == 0))
        check_labels(gpu, g, name="er%d" % t)


def test_degenerate_graphs(gpu):
    # isolated vertices, a single vertex, self loops only, one big cycle, a DAG path
    check_labels(gpu, graphgen.from_arcs(1, [], []), name="n1")
    check_labels(gpu, graphgen.from_arcs(5, [], []), name="n5_noarcs")
    check_labels(gpu, graphgen.from_arcs(4, [0, 1, 2, 3], [0, 1, 2, 3]), name="selfloops")
    n = 5000
    check_labels(gpu, graphgen.from_arcs(n, np.arange(n), (np.arange(n) + 1) % n), name="cycle5000")
    check_labels(gpu, graphgen.from_arcs(n, np.arange(n - 1), np.arange(1, n)), name="path5000")
    # parallel arcs
    check_labels(gpu, graphgen.from_arcs(3, [0, 0, 1, 2, 2], [1, 1, 2, 0, 0]), name="multiarcs")


@pytest.mark.parametrize("opt", [dict(), dict(table_floor=0.0, table_init=1024), dict(beta=8.0)])
def test_quadratic_reach(gpu, opt):
    # m 2-cycles (a_i, b_i) with arcs a_i -> a_j for every i < j: each source
    # reaches every later cycle in one hop, so a batch of k sources puts about
    # k*m/2 pairs into its first round's frontier, far above the vertex count;
    # reach tables and frontier buffers overflow and the searches restart
    m = 400
    i, j = np.triu_indices(m, 1)
    src = np.concatenate([np.arange(m), np.arange(m) + m, i])
    dst = np.concatenate([np.arange(m) + m, np.arange(m), j])
    g = graphgen.from_arcs(2 * m, src, dst)
    st = check_labels(gpu, g, gpu.default_options(**opt), name="cycle-dag m=%d %s" % (m, opt))
    assert st["restart_rounds"] <= st["rounds_multi"]


@pytest.mark.parametrize("first,packed", [(0, 0), (1, 0), (1, 1)])
def test_first_slot_families(gpu, first, packed):
    # the inline first-source slot (separate or in packed records) on every
    # family, including pair-heavy batches (the quadratic-reach graph) and
    # restarts on a tiny table
    opts = gpu.default_options(first_slot=first, packed=packed)
    for g in (graphgen.rmat(13, 16, seed=61), graphgen.knn(40000, 4, 5, 0.01, seed=62),
              graphgen.grid(150, 160, 0.5, seed=63), graphgen.lattice_oriented(60, 70, 1, seed=64)):
        check_labels(gpu, g, opts, name="%s first_slot=%d" % (g.name, first))
    m = 300
    i, j = np.triu_indices(m, 1)
    g = graphgen.from_arcs(2 * m, np.concatenate([np.arange(m), np.arange(m) + m, i]),
                           np.concatenate([np.arange(m) + m, np.arange(m), j]))
    check_labels(gpu, g, gpu.default_options(first_slot=first, packed=packed, beta=8.0),
                 name="cycle-dag first_slot=%d packed=%d" % (first, packed))
    n = 20000
    g = graphgen.from_arcs(n, np.arange(n - 1), np.arange(1, n))
    st = check_labels(gpu, g, gpu.default_options(first_slot=first, packed=packed, table_init=1024, table_floor=0.0),
                      name="path20000 small table first_slot=%d packed=%d" % (first, packed))
    if not first:
        assert st["table_restarts"] > 0


def test_graph_rounds_replays_match_the_oracle(gpu):
    # blocks of sparse rounds as captured HIP graphs: every call replays the
    # cached graphs, with the library's own eager launches and host checks
    # between replays; each call's labels must stay exact
    opts = gpu.default_options(graph_rounds=1)
    for g in (graphgen.grid(300, 300, 0.5, seed=65), graphgen.knn(60000, 6, 5, 0.01, seed=66),
              graphgen.rmat(14, 8, seed=67)):
        for rep in range(3):
            check_labels(gpu, g, opts, name="%s graph_rounds rep %d" % (g.name, rep))
    check_labels(gpu, graphgen.from_arcs(20000, np.arange(19999), np.arange(1, 20000)),
                 gpu.default_options(graph_rounds=1, table_init=1024, table_floor=0.0, first_slot=0),
                 name="path20000 graph_rounds restarts")


def test_forced_small_table_restarts(gpu):
    # a path: the first search splits it into two long subproblems, so the
    # next batch's sources reach thousands of vertices in some direction,
    # far more than a 1024-slot table holds
    n = 20000
    g = graphgen.from_arcs(n, np.arange(n - 1), np.arange(1, n))
    # (pairs in the table only: first-source slots would take the first pair of every vertex)
    st = check_labels(gpu, g, gpu.default_options(table_init=1024, table_floor=0.0, first_slot=0),
                      name="path20000 small table")
    assert st["table_restarts"] > 0


@pytest.mark.parametrize("first,packed", [(1, -1), (0, 0)])
def test_fast_grown_batch_is_retaken(gpu, first, packed):
    # an R-MAT graph of the 4096-graph batch (scale 15, edge factor 8): after
    # cheap batches the next one grows 64x into the large subproblem left by
    # the first SCC, and its pairs outgrow the tables; the batch is abandoned
    # and retaken at beta growth (before, its tables restarted a dozen times
    # over about 6.9 million claims)
    g = graphgen.batched_slice(4096, 1004, 3.0, 6.0, 1770, 1771)[0]
    assert g.n == 32768
    st = check_labels(gpu, g, gpu.default_options(first_slot=first, packed=packed),
                      name="%s first=%d packed=%d" % (g.name, first, packed))
    assert st["table_restarts"] >= 1
    assert st["claims"] < 20 * g.n


def test_hub_pass_with_and_without_heavy_vertices(gpu):
    # the edge-parallel pass over hub lists is skipped once a check has seen
    # that no vertex has more than 1024 arcs; alternate calls on one context
    # between graphs with and without such vertices (a stale degree maximum
    # would drop the hubs' arcs)
    n = 6000
    hub = graphgen.from_arcs(n, np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n), np.arange(1, n - 1)]),
                             np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64), np.arange(2, n)]))
    one_way = graphgen.from_arcs(n, np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n - 1)]),
                                 np.concatenate([np.arange(1, n), np.arange(2, n)]))
    lattice = graphgen.grid(120, 130, 0.5, seed=91)
    for rep in range(2):
        for g, name in ((hub, "wheel"), (lattice, "grid"), (one_way, "fan"), (graphgen.rmat(12, 16, seed=92), "rmat")):
            for opts in (gpu.default_options(), gpu.default_options(tau=1, dense=0), gpu.default_options(graph_rounds=1)):
                check_labels(gpu, g, opts, name="%s rep %d" % (name, rep))


def test_empty_graph(gpu):
    import torch
    say("empty graph")
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    dg = gpu.DeviceGraph(0, 0, z, e, z, e)
    assert gpu.scc_labels(dg).numel() == 0


@pytest.mark.parametrize("which", ["torus64", "grid200", "rmat12", "knn20k", "er_dense"])
def test_families_small(gpu, which):
    g = {"torus64": lambda: graphgen.torus(64, 64, 0.5, seed=1),
         "grid200": lambda: graphgen.grid(200, 200, 0.5, seed=2),
         "rmat12": lambda: graphgen.rmat(12, 16, seed=3),
         "knn20k": lambda: graphgen.knn(20000, 2, 5, 0.01, seed=4),
         "er_dense": lambda: graphgen.random_digraph(3000, 6.0, seed=5)}[which]()
    check_labels(gpu, g)


def test_config0_full_size(gpu):
    st = check_labels(gpu, graphgen.config(0))
    assert st["batches"] > 1 and st["trimmed"] > 0


@pytest.mark.parametrize("opt", [
    dict(tau=0), dict(tau=1), dict(tau=4), dict(tau=512, lambda_log2=10), dict(tau=65536),
    dict(seeds_per_wave=1), dict(seeds_per_wave=64),
    dict(beta=1.1), dict(beta=1.5), dict(beta=8.0), dict(beta_fast=0.0), dict(beta_fast=64.0), dict(arcs_per_lane=1), dict(arcs_per_lane=2),
    dict(arcs_per_lane=1, tau=512, lambda_log2=10),
    dict(lambda_log2=6, sigma=1, kappa=0),
    dict(table_init=1024), dict(trim=0), dict(seed=12345), dict(table_floor=0.0), dict(table_floor=0.3),
    dict(first_slot=1), dict(first_slot=1, tau=1), dict(first_slot=1, table_init=1024, table_floor=0.0),
    dict(first_slot=1, arcs_per_lane=2), dict(vgc_measure=1), dict(vgc_measure=1, tau=64, first_slot=1),
    dict(packed=1), dict(packed=0), dict(packed=1, table_init=1024, table_floor=0.0), dict(packed=1, tau=1),
    dict(packed=1, arcs_per_lane=4), dict(packed=1, graph_rounds=1),
    dict(tau_single=1), dict(tau_single=64), dict(tau_single=65536, tau=1),
])
def test_schedule_invariance(gpu, opt):
    g = graphgen.torus(100, 120, 0.55, seed=77)
    check_labels(gpu, g, gpu.default_options(**opt), name="torus100x120 %s" % opt)


def test_rounds_vgc_not_more_than_bfs(gpu):
    # with tau <= 1 a search takes one round per BFS level; local search can only merge rounds
    g = graphgen.grid(150, 150, 0.7, seed=8)
    say("rounds grid150")
    dg = gpu.to_device(g)
    _, plain = gpu.scc_labels(dg, gpu.default_options(tau=1, seed=3), return_stats=True)
    _, vgc = gpu.scc_labels(dg, gpu.default_options(tau=512, seed=3), return_stats=True)
    assert vgc["rounds_first"] <= plain["rounds_first"]
    assert vgc["rounds_first"] + vgc["rounds_multi"] <= plain["rounds_first"] + plain["rounds_multi"]


def test_reach_rounds_equal_bfs_levels_without_vgc(gpu):
    # Algorithm 2: with tau <= 1 (no local search) a search runs one frontier
    # round per BFS level, so its rounds are the largest BFS depth of its
    # sources plus one (the last round finds nothing); local search can only
    # merge rounds
    rng = np.random.default_rng(31)
    graphs = [graphgen.grid(60, 70, 0.7, seed=41), graphgen.torus(50, 50, 0.55, seed=42),
              graphgen.from_arcs(3000, np.arange(2999), np.arange(1, 3000)), graphgen.rmat(11, 8, seed=43),
              graphgen.knn(20000, 4, 5, 0.01, seed=44)]
    for g in graphs:
        dg = gpu.to_device(g)
        labels = np.zeros(g.n, np.int32)
        if g.n > 5000:
            labels[rng.random(g.n) < 0.1] = -1
        cand = np.nonzero(labels >= 0)[0]
        for k in (1, 3, 40):
            src = rng.permutation(cand)[:k].astype(np.int32)
            for d in (0, 1):
                off, adj = (g.out_off, g.out_adj) if d == 0 else (g.in_off, g.in_adj)
                depth = int(oracle.bfs_depths(g.n, off, adj, labels, src).max())
                key = "rounds_first" if k == 1 else "rounds_multi"
                for dense in ((0, 1) if k == 1 else (0,)):
                    say("rounds", g.name, "k", k, "dir", d, "dense", dense)
                    # a table large enough for every pair: no restart, so the
                    # round count covers the whole search
                    big = 1 << int(np.ceil(np.log2(2 * k * g.n + 1024)))
                    got, st = gpu.scc_reach(dg, src, labels, direction=d, return_stats=True,
                                            options=gpu.default_options(tau=1, dense=dense, table_init=big))
                    assert st["table_restarts"] == 0
                    assert st[key] == depth + 1, (g.name, k, d, dense, st[key], depth)
                    want = oracle.reach_pairs(g.n, off, adj, labels, src)
                    assert np.array_equal(as_pairs(got.cpu().numpy()), want)
                _, st = gpu.scc_reach(dg, src, labels, direction=d, return_stats=True,
                                      options=gpu.default_options(tau=2048))
                assert st[key] <= depth + 1


def test_reach_matches_oracle(gpu):
    rng = np.random.default_rng(1)
    for t, g in enumerate([graphgen.torus(40, 40, 0.6, seed=3), graphgen.rmat(10, 8, seed=4),
                           graphgen.random_digraph(500, 1.5, seed=6)]):
        dg = gpu.to_device(g)
        for trial in range(3):
            labels = rng.integers(-1, 3, size=g.n).astype(np.int32)
            if trial == 0:
                labels[:] = 0
            cand = np.nonzero(labels >= 0)[0]
            for k in (1, 2, 17):
                src = rng.permutation(cand)[:k].astype(np.int32)
                for d in (0, 1):
                    say("reach", g.name, "trial", trial, "k", k, "dir", d)
                    got = gpu.scc_reach(dg, src, labels, direction=d).cpu().numpy()
                    off, adj = (g.out_off, g.out_adj) if d == 0 else (g.in_off, g.in_adj)
                    want = oracle.reach_pairs(g.n, off, adj, labels, src)
                    assert np.array_equal(as_pairs(got), want)


def test_reach_rejects_bad_sources(gpu):
    g = graphgen.torus(10, 10, 0.6, seed=3)
    dg = gpu.to_device(g)
    lab = np.zeros(g.n, np.int32)
    lab[4] = -1
    say("reach errors")
    with pytest.raises(gpu.SccError):
        gpu.scc_reach(dg, [4], lab)          # excluded source
    with pytest.raises(gpu.SccError):
        gpu.scc_reach(dg, [1, 1], lab)       # duplicate
    with pytest.raises(gpu.SccError):
        gpu.scc_reach(dg, [100], lab)        # out of range
    assert gpu.scc_reach(dg, [], lab).shape[0] == 0
    # the context still works after errors
    got = gpu.scc_reach(dg, [0], np.zeros(g.n, np.int32)).cpu().numpy()
    want = oracle.reach_pairs(g.n, g.out_off, g.out_adj, np.zeros(g.n, np.int32), [0])
    assert np.array_equal(as_pairs(got), want)


def test_invalid_graph_rejected(gpu):
    import torch
    say("invalid graphs")
    g = graphgen.torus(8, 8, 0.6, seed=3)
    dg = gpu.to_device(g)
    bad = gpu.DeviceGraph(dg.n, dg.m, dg.out_off.clone(), dg.out_adj.clone(), dg.in_off, dg.in_adj)
    bad.out_adj[3] = g.n + 5
    with pytest.raises(gpu.SccError) as e:
        gpu.scc_labels(bad)
    assert e.value.code == -2
    bad = gpu.DeviceGraph(dg.n, dg.m, dg.out_off.clone(), dg.out_adj, dg.in_off, dg.in_adj)
    bad.out_off[5] = bad.out_off[6] + 1
    with pytest.raises(gpu.SccError):
        gpu.scc_labels(bad)
    bad = gpu.DeviceGraph(dg.n, dg.m, dg.out_off, dg.out_adj, dg.in_off, torch.roll(dg.in_adj, 1))
    # a rolled in_adj keeps degrees only by accident; in-degree histogram differs here
    if not np.array_equal(np.bincount(g.out_adj, minlength=g.n), np.diff(g.in_off)):
        with pytest.raises(gpu.SccError):
            gpu.scc_labels(bad)
    check_labels(gpu, g, name="after errors")


def test_hash_bag_extract_is_inserted_multiset(gpu):
    import torch
    rng = np.random.default_rng(0)
    for n, rounds, lam in [(1, 1, 10), (1000, 1, 10), (100000, 3, 6), (300000, 1, 10), (50000, 7, 8)]:
        say("bag", n, rounds, lam)
        keys = rng.integers(0, 1 << 62, size=n).astype(np.int64)
        keys[: n // 10] = keys[0]  # duplicates must all survive (no dedupe)
        out, st = gpu.bag_selftest(torch.from_numpy(keys).cuda(), rounds,
                                   gpu.default_options(lambda_log2=lam), return_stats=True)
        got = np.sort(out.cpu().numpy())
        assert np.array_equal(got, np.sort(np.concatenate(oracle.hashbag_model(
            [keys[r::rounds] for r in range(rounds)]))))
        if n >= 100000:
            assert st["bag_chunk_advances"] > 0


def test_hash_bag_theorem1_load_and_prefix(gpu):
    # Theorem 1 / Appendix A with alpha = 1/2: a chunk is left at a load in
    # [1/4, 3/4] w.h.p. once chunks are large against the inserts in flight
    # (k = Omega(P sigma): here 4096 wavefronts of 64 against chunks of 2^22),
    # and s elements occupy the first O(s + lambda) slots
    import torch
    loads, forced = [], []
    for seed in range(20):
        s = 12_000_000 + 500_000 * seed
        keys = torch.arange(s, dtype=torch.int64, device="cuda") * 2654435761 + seed
        say("bag theorem1 seed", seed, "s", s)
        opts = gpu.default_options(lambda_log2=22, sigma=50, alpha=0.5, seed=seed + 1)
        out = gpu.bag_selftest(keys, 1, opts)
        assert out.numel() == s
        rows, prefix = gpu.bag_stats()
        loads += [r[2] for r in rows if r[3] == 0]
        forced += [r[2] for r in rows if r[3] == 1]
        assert len(prefix) == 1 and prefix[0] <= 8 * (s + (1 << 22)), (prefix, s)
    say("bag loads at a move: sampled", np.round(sorted(loads), 3), "probe limit", np.round(sorted(forced), 3))
    assert loads, "no chunk was left by its samples"
    assert min(loads) >= 0.25 and max(loads) <= 0.75, (min(loads), max(loads))
    # the probe limit is the rare fallback; a chunk it ends is still well used
    assert len(forced) <= 0.2 * (len(loads) + len(forced)) and all(x >= 0.125 for x in forced)


def test_bag_lambda_change_on_one_context(gpu):
    # a small first chunk on one call, the automatic one on the next: each
    # search lane keeps a chunk count that fits its own buffers
    g = graphgen.knn(60000, 6, 5, 0.01, seed=45)
    check_labels(gpu, g, gpu.default_options(lambda_log2=6), name="knn60k lambda 2^6")
    check_labels(gpu, g, gpu.default_options(), name="knn60k lambda auto")
    check_labels(gpu, g, gpu.default_options(lambda_log2=6), name="knn60k lambda 2^6 again")


def test_batched_matches_per_graph_oracle(gpu):
    import torch
    graphs = graphgen.batched(24, seed=77, lo_exp=1.5, hi_exp=3.5) + [graphgen.from_arcs(0, [], []),
                                                                      graphgen.from_arcs(3, [0], [1])]
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    say("batched", len(graphs), "graphs", int(vb[-1]), "vertices")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    got = gpu.scc_labels_batched(vb, ab, t(oo), t(oa), t(io), t(ia)).cpu().numpy()
    for i, g in enumerate(graphs):
        want = oracle.scc_graph(g)
        assert np.array_equal(got[vb[i]:vb[i + 1]], want), "graph %d" % i


def test_policy_kernel_matches_cpu_forward(gpu):
    rng = np.random.default_rng(5)
    w = (rng.standard_normal(gpu.POLICY_FLOATS) * 0.3).astype(np.float32)
    x = rng.standard_normal((33, 5)).astype(np.float32)
    say("policy eval")
    gpu.policy_load(w)
    got = gpu.policy_eval(x)
    want = oracle.policy_forward(w, x)
    assert np.allclose(got, want, rtol=1e-5, atol=1e-5)
    bad = w.copy()
    bad[7] = np.nan
    with pytest.raises(gpu.SccError):
        gpu.policy_load(bad)


@pytest.mark.parametrize("dense", [-1, 0, 1])
def test_dense_mode_invariance(gpu, dense):
    for g in (graphgen.rmat(13, 16, seed=11), graphgen.torus(80, 80, 0.6, seed=12),
              graphgen.knn(30000, 3, 5, 0.01, seed=13)):
        st = check_labels(gpu, g, gpu.default_options(dense=dense), name="%s dense=%d" % (g.name, dense))
        if dense == 1:
            assert st["dense_rounds"] > 0
        if dense == 0:
            assert st["dense_rounds"] == 0


def test_dense_reach_matches_oracle(gpu):
    g = graphgen.rmat(12, 16, seed=14)
    dg = gpu.to_device(g)
    lab = np.zeros(g.n, np.int32)
    for dense in (1, -1):
        for d in (0, 1):
            say("dense reach", dense, d)
            got = gpu.scc_reach(dg, [int(np.argmax(np.diff(g.out_off)))], lab, direction=d,
                                options=gpu.default_options(dense=dense)).cpu().numpy()
            off, adj = (g.out_off, g.out_adj) if d == 0 else (g.in_off, g.in_adj)
            want = oracle.reach_pairs(g.n, off, adj, lab, [int(np.argmax(np.diff(g.out_off)))])
            assert np.array_equal(as_pairs(got), want)


def test_policy_and_exploration_do_not_change_labels(gpu):
    rng = np.random.default_rng(9)
    g = graphgen.knn(50000, 5, 5, 0.01, seed=21)
    w = (rng.standard_normal(gpu.POLICY_FLOATS) * 0.5).astype(np.float32)
    gpu.policy_load(w)
    st = check_labels(gpu, g, gpu.default_options(policy=1), name="knn50k learned(random weights)")
    assert st["policy_calls"] > 0
    st = check_labels(gpu, g, gpu.default_options(policy=2, trace=1), name="knn50k explore+trace")
    rows = gpu.trace_read()
    assert rows.shape[1] == gpu.TRACE_FIELDS and len(rows) == st["rounds_first"] + st["rounds_multi"]
    assert set(np.unique(rows[:, 6])) <= {512.0, 1024.0, 2048.0, 4096.0}
    check_labels(gpu, graphgen.rmat(13, 16, seed=22), gpu.default_options(policy=1, dense=-1), name="rmat13 learned")
