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


def sorted_pairs(p):
    p = np.asarray(p).reshape(-1, 2)
    return p[np.lexsort((p[:, 0], p[:, 1]))]


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
    check_labels(gpu, g, gpu.default_options(**opt), name="cycle-dag m=%d %s" % (m, opt))


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
])
def test_schedule_invariance(gpu, opt):
    g = graphgen.torus(100, 120, 0.55, seed=77)
    st = check_labels(gpu, g, gpu.default_options(**opt), name="torus100x120 %s" % opt)
    if opt.get("table_init") == 1024:
        assert st["table_restarts"] >= 0


def test_rounds_vgc_not_more_than_bfs(gpu):
    # with tau <= 1 a search takes one round per BFS level; local search can only merge rounds
    g = graphgen.grid(150, 150, 0.7, seed=8)
    say("rounds grid150")
    dg = gpu.to_device(g)
    _, plain = gpu.scc_labels(dg, gpu.default_options(tau=1, seed=3), return_stats=True)
    _, vgc = gpu.scc_labels(dg, gpu.default_options(tau=512, seed=3), return_stats=True)
    assert vgc["rounds_first"] <= plain["rounds_first"]
    assert vgc["rounds_first"] + vgc["rounds_multi"] <= plain["rounds_first"] + plain["rounds_multi"]


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
                    assert np.array_equal(sorted_pairs(got), want)


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
    assert np.array_equal(sorted_pairs(got), want)


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
        assert np.array_equal(got, oracle.hashbag_model([keys])[0])
        if n >= 100000:
            assert st["bag_chunk_advances"] > 0


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
            assert np.array_equal(sorted_pairs(got), want)


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
