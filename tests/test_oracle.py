"""Pins for the sequential oracle (CPU only).

The oracle is checked against things other than itself: brute-force closure
on every digraph with n <= 4, random tiny graphs, closed forms (cycles, DAGs,
complete digraphs, lattices with p = 1), an independent library routine
(SciPy's strong/weak connected components), and the certificate checker,
which in turn is shown to reject planted mistakes.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle
from tests import brute


def csr_of(n, arcs):
    src = np.array([a for a, _ in arcs], dtype=np.int32)
    dst = np.array([b for _, b in arcs], dtype=np.int32)
    return graphgen.from_arcs(n, src, dst)


def scipy_min_labels(g):
    A = sp.csr_matrix((np.ones(g.m), g.out_adj, g.out_off), shape=(g.n, g.n))
    _, comp = connected_components(A, directed=True, connection="strong")
    mins = np.full(comp.max() + 1 if g.n else 0, g.n, np.int64)
    np.minimum.at(mins, comp, np.arange(g.n))
    return mins[comp].astype(np.int32)


def all_pairs(n, loops):
    return [(u, v) for u in range(n) for v in range(n) if loops or u != v]


@pytest.mark.parametrize("n,loops", [(1, True), (2, True), (3, True), (4, False)])
def test_tarjan_exhaustive_tiny(n, loops):
    cand = all_pairs(n, loops)
    for mask in range(1 << len(cand)):
        arcs = [cand[i] for i in range(len(cand)) if mask >> i & 1]
        g = csr_of(n, arcs)
        got = oracle.scc_graph(g)
        want = brute.scc_min_labels(n, g.out_off, g.out_adj)
        assert np.array_equal(got, want), (n, arcs)


def test_tarjan_random_small_vs_brute():
    rng = np.random.default_rng(7)
    for t in range(250):
        n = int(rng.integers(1, 120))
        d = float(rng.choice([0.5, 1.0, 1.5, 2.5, 5.0]))
        g = graphgen.random_digraph(n, d, seed=5000 + t, self_loops=bool(t % 3 == 0))
        got = oracle.scc_graph(g)
        assert np.array_equal(got, brute.scc_min_labels(n, g.out_off, g.out_adj))
        assert oracle.check_partition(g, got) == (0, -1)


@pytest.mark.parametrize("seed", range(6))
def test_tarjan_vs_scipy_medium(seed):
    for g in (graphgen.random_digraph(3000, 1.2 + 0.3 * seed, seed=seed),
              graphgen.torus(40 + seed, 50, 0.5, seed=seed),
              graphgen.rmat(11, 8, seed=seed),
              graphgen.knn(4000, 4, 5, 0.01, seed=seed)):
        got = oracle.scc_graph(g)
        assert np.array_equal(got, scipy_min_labels(g)), g.name
        assert oracle.check_partition(g, got) == (0, -1)


def test_closed_forms():
    # directed n-cycle: one SCC
    n = 1000
    g = csr_of(n, [(i, (i + 1) % n) for i in range(n)])
    assert (oracle.scc_graph(g) == 0).all()
    # DAG (arcs i -> j only for i < j): n singletons
    rng = np.random.default_rng(1)
    arcs = set()
    while len(arcs) < 3000:
        a, b = sorted(rng.integers(0, n, 2))
        if a != b:
            arcs.add((int(a), int(b)))
    g = csr_of(n, sorted(arcs))
    assert np.array_equal(oracle.scc_graph(g), np.arange(n))
    # complete digraph: one SCC
    g = csr_of(30, all_pairs(30, False))
    assert (oracle.scc_graph(g) == 0).all()
    # full torus (p = 1): one SCC; grid with only right/down arcs: singletons
    g = graphgen.torus(37, 41, 1.0, seed=3)
    assert (oracle.scc_graph(g) == 0).all()
    r, c = 30, 20
    arcs = [(i * c + j, i * c + j + 1) for i in range(r) for j in range(c - 1)]
    arcs += [(i * c + j, (i + 1) * c + j) for i in range(r - 1) for j in range(c)]
    g = csr_of(r * c, arcs)
    assert np.array_equal(oracle.scc_graph(g), np.arange(r * c))
    # empty graph and isolated vertices
    assert len(oracle.scc_labels(0, np.zeros(1, np.int32), np.zeros(0, np.int32))) == 0
    g = csr_of(5, [])
    assert np.array_equal(oracle.scc_graph(g), np.arange(5))


def test_symmetric_digraph_scc_equals_undirected_cc():
    for seed in range(4):
        base = graphgen.random_digraph(4000, 0.7, seed=100 + seed)
        src = np.repeat(np.arange(base.n), np.diff(base.out_off)).astype(np.int32)
        dst = base.out_adj
        g = graphgen.from_arcs(base.n, np.concatenate([src, dst]), np.concatenate([dst, src]), dedup=True)
        A = sp.csr_matrix((np.ones(base.m), base.out_adj, base.out_off), shape=(base.n, base.n))
        _, comp = connected_components(A, directed=True, connection="weak")
        mins = np.full(comp.max() + 1, base.n)
        np.minimum.at(mins, comp, np.arange(base.n))
        assert np.array_equal(oracle.scc_graph(g), mins[comp])


def test_self_loops_do_not_change_sccs():
    g = graphgen.random_digraph(500, 1.3, seed=11)
    base = oracle.scc_graph(g)
    src = np.repeat(np.arange(g.n), np.diff(g.out_off)).astype(np.int32)
    loops = np.arange(0, g.n, 3, dtype=np.int32)
    g2 = graphgen.from_arcs(g.n, np.concatenate([src, loops]), np.concatenate([g.out_adj, loops]))
    assert np.array_equal(oracle.scc_graph(g2), base)


def test_check_partition_rejects_planted_mistakes():
    g = graphgen.torus(30, 30, 0.5, seed=9)
    lab = oracle.scc_graph(g)
    assert oracle.check_partition(g, lab) == (0, -1)
    # merge two distinct SCCs that are joined by an arc: not strongly connected
    comps, sizes = np.unique(lab, return_counts=True)
    big = comps[np.argmax(sizes)]
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    cross = [(u, w) for u, w in zip(src, g.out_adj) if lab[u] != lab[w]]
    u, w = cross[0]
    bad = lab.copy()
    a, b = sorted((lab[u], lab[w]))
    bad[bad == b] = a
    assert oracle.check_partition(g, bad)[0] == 1
    # split the largest SCC in two: the class graph gets a cycle or a class
    # loses strong connectivity
    bad = lab.copy()
    members = np.nonzero(lab == big)[0]
    second = members[len(members) // 2:]
    bad[second] = second.min()
    assert oracle.check_partition(g, bad)[0] in (1, 2)
    # a label that is not the class minimum
    bad = lab.copy()
    bad[members] = members.max()
    assert oracle.check_partition(g, bad)[0] == 3


def test_reach_pairs_vs_brute():
    rng = np.random.default_rng(3)
    for t in range(150):
        n = int(rng.integers(1, 60))
        g = graphgen.random_digraph(n, float(rng.choice([0.8, 1.5, 3.0])), seed=7000 + t)
        labels = rng.integers(-1, 3, size=n).astype(np.int32)
        cand = np.nonzero(labels >= 0)[0]
        if len(cand) == 0:
            continue
        k = int(rng.integers(1, len(cand) + 1))
        sources = rng.permutation(cand)[:k].astype(np.int32)
        got = oracle.reach_pairs(n, g.out_off, g.out_adj, labels, sources)
        want = brute.reach_pairs(n, g.out_off, g.out_adj, labels, sources)
        assert np.array_equal(got, want)
        # backward search = forward search on the transpose
        got_b = oracle.reach_pairs(n, g.in_off, g.in_adj, labels, sources)
        R = brute.closure(n, g.out_off, g.out_adj, lambda u, w: labels[u] == labels[w] and labels[u] >= 0)
        want_b = [(int(v), j) for j, s in enumerate(sources) for v in np.nonzero(R[:, s])[0]]
        assert np.array_equal(got_b, np.array(want_b, np.int32).reshape(-1, 2))


def test_reach_pairs_special_cases():
    g = graphgen.torus(25, 25, 0.6, seed=4)
    labels = np.zeros(g.n, np.int32)
    # all labels equal, one source: the plain BFS reach set (scipy)
    from scipy.sparse.csgraph import breadth_first_order
    A = sp.csr_matrix((np.ones(g.m), g.out_adj, g.out_off), shape=(g.n, g.n))
    order = breadth_first_order(A, 17, directed=True, return_predecessors=False)
    got = oracle.reach_pairs(g.n, g.out_off, g.out_adj, labels, [17])
    assert np.array_equal(got[:, 0], np.sort(order)) and (got[:, 1] == 0).all()
    # excluded source and duplicate source are rejected
    labels2 = labels.copy()
    labels2[5] = -1
    with pytest.raises(ValueError):
        oracle.reach_pairs(g.n, g.out_off, g.out_adj, labels2, [5])
    with pytest.raises(ValueError):
        oracle.reach_pairs(g.n, g.out_off, g.out_adj, labels, [3, 3])
    # no sources: empty
    assert oracle.reach_pairs(g.n, g.out_off, g.out_adj, labels, []).shape == (0, 2)
    # symmetric graph: the reach set of s is its connected component
    base = graphgen.random_digraph(800, 0.8, seed=21)
    src = np.repeat(np.arange(base.n), np.diff(base.out_off)).astype(np.int32)
    sym = graphgen.from_arcs(base.n, np.concatenate([src, base.out_adj]), np.concatenate([base.out_adj, src]),
                             dedup=True)
    A = sp.csr_matrix((np.ones(base.m), base.out_adj, base.out_off), shape=(base.n, base.n))
    _, comp = connected_components(A, directed=True, connection="weak")
    got = oracle.reach_pairs(sym.n, sym.out_off, sym.out_adj, np.zeros(sym.n, np.int32), [0, 400])
    for j, s in enumerate([0, 400]):
        assert np.array_equal(got[got[:, 1] == j, 0], np.nonzero(comp == comp[s])[0])


def test_policy_forward_matches_manual():
    rng = np.random.default_rng(0)
    n_in, hid, n_out = 5, 32, 8
    w = rng.standard_normal(hid * n_in + hid + hid * hid + hid + n_out * hid + n_out).astype(np.float32)
    x = rng.standard_normal((4, n_in)).astype(np.float32)
    y = oracle.policy_forward(w, x)
    # element by element in float64, then compare within float32 rounding
    o = 0
    W1 = w[o:o + hid * n_in].reshape(hid, n_in).astype(np.float64); o += hid * n_in
    b1 = w[o:o + hid].astype(np.float64); o += hid
    W2 = w[o:o + hid * hid].reshape(hid, hid).astype(np.float64); o += hid * hid
    b2 = w[o:o + hid].astype(np.float64); o += hid
    W3 = w[o:o + n_out * hid].reshape(n_out, hid).astype(np.float64); o += n_out * hid
    b3 = w[o:o + n_out].astype(np.float64)
    for r in range(4):
        h1 = [max(0.0, sum(W1[i, j] * x[r, j] for j in range(n_in)) + b1[i]) for i in range(hid)]
        h2 = [max(0.0, sum(W2[i, j] * h1[j] for j in range(hid)) + b2[i]) for i in range(hid)]
        out = [sum(W3[i, j] * h2[j] for j in range(hid)) + b3[i] for i in range(n_out)]
        assert np.allclose(y[r], out, rtol=1e-4, atol=1e-4)


def test_hashbag_model_is_multiset_identity():
    batches = [[5, 1, 5, 3], [], [2]]
    out = oracle.hashbag_model(batches)
    assert [list(b) for b in out] == [[1, 3, 5, 5], [], [2]]


# ---------------------------------------------------------------- policy ----
# Closed forms for the MLP forward, built from the documented blob layout
# [W1 (32 x 5), b1 (32), W2 (32 x 32), b2 (32), W3 (8 x 32), b3 (8)], row-major
# out x in.  None of them recomputes the forward with matrix products: each
# predicts the output from the layout alone, so a transposed block, a wrong
# offset, a dropped bias or ReLU fails one of them.
N_IN, HID, N_OUT = 5, 32, 8
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * N_IN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + N_OUT * HID
N_W = OFF_B3 + N_OUT


def _identity_net():
    """h1 = 1 for every hidden unit (W1 = 0, b1 = 1), h2 = h1 (W2 = I),
    y[o] = h2[o] (W3 row o picks hidden unit o), b3 = 0: y = 1 everywhere."""
    w = np.zeros(N_W, np.float32)
    w[OFF_B1:OFF_B1 + HID] = 1.0
    for i in range(HID):
        w[OFF_W2 + i * HID + i] = 1.0
    for o in range(N_OUT):
        w[OFF_W3 + o * HID + o] = 1.0
    return w


def test_policy_forward_one_hot_copies_inputs():
    # W1 row i (i < 5) = e_i, W2 = I, W3 row o = e_o: y[o] = relu(x[o]) for
    # o < 5 and y[o] = b3[o] for the other outputs
    w = np.zeros(N_W, np.float32)
    for i in range(N_IN):
        w[OFF_W1 + i * N_IN + i] = 1.0
    for i in range(HID):
        w[OFF_W2 + i * HID + i] = 1.0
    for o in range(N_OUT):
        w[OFF_W3 + o * HID + o] = 1.0
    w[OFF_B3:OFF_B3 + N_OUT] = [0, 0, 0, 0, 0, 7.5, -2.25, 0.125]
    x = np.array([[1.5, -2.0, 3.25, 0.0, 9.0], [-1, -1, -1, -1, -1]], np.float32)
    y = oracle.policy_forward(w, x)
    assert np.array_equal(y[0], np.array([1.5, 0.0, 3.25, 0.0, 9.0, 7.5, -2.25, 0.125], np.float32))
    assert np.array_equal(y[1], np.array([0, 0, 0, 0, 0, 7.5, -2.25, 0.125], np.float32))


def test_policy_forward_dead_relus_give_b3():
    # every pre-activation of both hidden layers negative: the output is b3 exactly
    rng = np.random.default_rng(11)
    w = (rng.standard_normal(N_W) * 0.01).astype(np.float32)
    w[OFF_B1:OFF_B1 + HID] = -100.0
    w[OFF_B2:OFF_B2 + HID] = -1.0
    x = rng.uniform(-3, 3, size=(16, N_IN)).astype(np.float32)
    y = oracle.policy_forward(w, x)
    assert np.array_equal(y, np.tile(w[OFF_B3:OFF_B3 + N_OUT], (16, 1)))


def _perturbation_prediction(f, x, delta):
    """Output change of _identity_net() when blob entry f grows by delta, from
    the layout: (block, row, column) of f decides which unit moves."""
    d = np.zeros(N_OUT)
    if f < OFF_B1:                       # W1[i, j]: h1[i] += delta * x[j]
        i, j = divmod(f - OFF_W1, N_IN)
        if i < N_OUT:
            d[i] = delta * x[j]
    elif f < OFF_W2:                     # b1[i]
        i = f - OFF_B1
        if i < N_OUT:
            d[i] = delta
    elif f < OFF_B2:                     # W2[i, j]: h2[i] += delta * h1[j] = delta
        i, _ = divmod(f - OFF_W2, HID)
        if i < N_OUT:
            d[i] = delta
    elif f < OFF_W3:                     # b2[i]
        i = f - OFF_B2
        if i < N_OUT:
            d[i] = delta
    elif f < OFF_B3:                     # W3[o, p]: y[o] += delta * h2[p] = delta
        o, _ = divmod(f - OFF_W3, HID)
        d[o] = delta
    else:                                # b3[o]
        d[f - OFF_B3] = delta
    return d


def _check_every_blob_offset(forward):
    x = np.array([1.0, 2.0, 3.0, 4.0, 5.0], np.float32)
    base = _identity_net()
    y0 = forward(base, x[None])[0].astype(np.float64)
    assert np.array_equal(y0, np.ones(N_OUT))
    bad = []
    for f in range(N_W):
        w = base.copy()
        w[f] += np.float32(0.5)
        dy = forward(w, x[None])[0].astype(np.float64) - y0
        if not np.allclose(dy, _perturbation_prediction(f, x, 0.5), rtol=0, atol=1e-6):
            bad.append(f)
    return bad


def test_policy_forward_blob_layout_every_offset():
    assert _check_every_blob_offset(oracle.policy_forward) == []


def test_policy_layout_pin_catches_transposed_w1():
    # the same check fails for a forward that reads W1 as (in x out)
    def transposed_w1(w, x):
        w2 = w.copy()
        w2[OFF_W1:OFF_B1] = w[OFF_W1:OFF_B1].reshape(N_IN, HID).T.reshape(-1)
        return oracle.policy_forward(w2, x)
    assert len(_check_every_blob_offset(transposed_w1)) > 0


# ------------------------------------------------------------ BFS depths ----
def test_bfs_depths_closed_forms():
    n = 300
    path = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    lab = np.zeros(n, np.int32)
    assert list(oracle.bfs_depths(n, path.out_off, path.out_adj, lab, [0, 100, n - 1])) == [n - 1, n - 1 - 100, 0]
    cyc = csr_of(n, [(i, (i + 1) % n) for i in range(n)])
    assert list(oracle.bfs_depths(n, cyc.out_off, cyc.out_adj, lab, [0, 5])) == [n - 1, n - 1]
    # right/down grid from the top-left corner: the Manhattan distance to the far corner
    r, c = 17, 23
    arcs = [(i * c + j, i * c + j + 1) for i in range(r) for j in range(c - 1)]
    arcs += [(i * c + j, (i + 1) * c + j) for i in range(r - 1) for j in range(c)]
    g = csr_of(r * c, arcs)
    assert oracle.bfs_depths(g.n, g.out_off, g.out_adj, np.zeros(g.n, np.int32), [0])[0] == r + c - 2
    # a label boundary cuts the path
    lab2 = np.zeros(n, np.int32)
    lab2[150:] = 1
    assert list(oracle.bfs_depths(n, path.out_off, path.out_adj, lab2, [0, 150])) == [149, n - 151]
    with pytest.raises(ValueError):
        lab3 = lab.copy()
        lab3[7] = -1
        oracle.bfs_depths(n, path.out_off, path.out_adj, lab3, [7])


def test_bfs_depths_vs_scipy_shortest_paths():
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(12)
    for t in range(40):
        g = graphgen.random_digraph(int(rng.integers(2, 400)), float(rng.choice([0.8, 1.5, 3.0])), seed=8100 + t)
        labels = rng.integers(-1, 2, size=g.n).astype(np.int32)
        cand = np.nonzero(labels >= 0)[0]
        if len(cand) == 0:
            continue
        src = rng.permutation(cand)[:5].astype(np.int32)
        u = np.repeat(np.arange(g.n), np.diff(g.out_off))
        keep = (labels[u] == labels[g.out_adj]) & (labels[u] >= 0)
        A = sp.csr_matrix((np.ones(int(keep.sum())), (u[keep], g.out_adj[keep])), shape=(g.n, g.n))
        D = shortest_path(A, method="D", directed=True, unweighted=True, indices=src)
        want = [int(np.max(D[j][np.isfinite(D[j])])) for j in range(len(src))]
        assert list(oracle.bfs_depths(g.n, g.out_off, g.out_adj, labels, src)) == want


# -------------------------------------------------------------- hash bag ----
def test_hashbag_model_returns_the_inserted_multiset():
    from collections import Counter
    rng = np.random.default_rng(4)
    batches = [[5, 1, 5, 3], [], [2], rng.integers(0, 50, size=20000), rng.integers(0, 1 << 40, size=70000)]
    sim = oracle.hashbag_sim(batches, lam_log2=8)
    for b, e in zip(batches, sim["extracted"]):
        assert Counter(np.asarray(b, np.int64).tolist()) == Counter(e.tolist())
    assert [list(x) for x in oracle.hashbag_model(batches[:3])] == [[1, 3, 5, 5], [], [2]]


@pytest.mark.parametrize("s", [3000, 40000, 250000])
def test_hashbag_model_theorem1_load_and_prefix(s):
    # Theorem 1 / Appendix A with alpha = 1/2: a chunk is left at load in
    # [1/4, 3/4] w.h.p., and s elements sit in the first O(s + lambda) slots
    lam = 1 << 10
    loads, moves = [], 0
    for seed in range(24):
        keys = np.arange(s, dtype=np.int64) * 7919 + seed
        sim = oracle.hashbag_sim([keys], lam_log2=10, sigma=50, alpha=0.5, kappa=32, seed=seed + 1)
        for chunk, load, cause in sim["advances"]:
            moves += 1
            if cause == 0:
                loads.append(load)
        assert sim["prefix"][0] <= 8 * (s + lam)
        assert sim["prefix"][0] >= s
    assert loads and all(0.25 <= x <= 0.75 for x in loads), (min(loads), max(loads))
    # the sample count, not the probe limit, moves the chunk almost always
    assert len(loads) >= 0.9 * moves


def test_hashbag_model_small_round_stays_in_first_chunk():
    sim = oracle.hashbag_sim([np.arange(64)] * 5, lam_log2=10)
    assert sim["advances"] == [] and list(sim["prefix"]) == [1024] * 5


def test_hashbag_load_pin_catches_a_wrong_sample_rate():
    # a model whose sample rate ignores alpha (rate sigma / size, i.e. alpha
    # near 1) leaves chunks nearly full: the Theorem 1 interval rejects it
    sim = oracle.hashbag_sim([np.arange(200000)], lam_log2=10, sigma=50, alpha=0.97, kappa=1 << 20, seed=3)
    loads = [ld for _, ld, cause in sim["advances"] if cause == 0]
    assert loads and max(loads) > 0.75


# ------------------------------------------------------ connected components ----
def test_wcc_vs_scipy_and_symmetric_scc():
    rng = np.random.default_rng(21)
    for t in range(30):
        n = int(rng.integers(1, 3000))
        g = graphgen.random_digraph(n, float(rng.choice([0.3, 0.8, 1.5])), seed=9100 + t)
        got = oracle.wcc_labels(g.n, g.out_off, g.out_adj)
        A = sp.csr_matrix((np.ones(g.m), g.out_adj, g.out_off), shape=(g.n, g.n))
        _, comp = connected_components(A, directed=True, connection="weak")
        mins = np.full(comp.max() + 1, g.n)
        np.minimum.at(mins, comp, np.arange(g.n))
        assert np.array_equal(got, mins[comp])
        # symmetrised: its SCCs (Tarjan) are its connected components
        src = np.repeat(np.arange(g.n), np.diff(g.out_off)).astype(np.int32)
        sym = graphgen.from_arcs(g.n, np.concatenate([src, g.out_adj]), np.concatenate([g.out_adj, src]), dedup=True)
        assert np.array_equal(oracle.wcc_labels(sym.n, sym.out_off, sym.out_adj), oracle.scc_graph(sym))


def test_wcc_closed_forms():
    n = 500
    path = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    assert (oracle.wcc_labels(n, path.out_off, path.out_adj) == 0).all()
    g = csr_of(6, [(5, 4), (2, 3)])
    assert list(oracle.wcc_labels(6, g.out_off, g.out_adj)) == [0, 1, 2, 2, 4, 4]
    assert len(oracle.wcc_labels(0, np.zeros(1, np.int32), np.zeros(0, np.int32))) == 0


# ----------------------------------------------------------------- LE-lists ----
def _le_by_definition(g, order):
    """u's list: walk the order, keep s when d(s, u) beats every earlier source."""
    from scipy.sparse.csgraph import shortest_path
    A = sp.csr_matrix((np.ones(g.m), g.out_adj, g.out_off), shape=(g.n, g.n))
    D = shortest_path(A, method="D", directed=True, unweighted=True)  # D[s, u]
    lists = []
    for u in range(g.n):
        best = np.inf
        row = []
        for s in order:
            if D[s, u] < best:
                best = D[s, u]
                row.append((int(s), int(D[s, u])))
        lists.append(row)
    return lists


def _le_rows(loff, src, dist, n):
    return [list(zip(src[loff[u]:loff[u + 1]].tolist(), dist[loff[u]:loff[u + 1]].tolist())) for u in range(n)]


def test_le_lists_vs_definition():
    rng = np.random.default_rng(23)
    for t in range(60):
        n = int(rng.integers(1, 90))
        g = graphgen.random_digraph(n, float(rng.choice([0.7, 1.5, 3.0])), seed=9300 + t)
        if t % 2:
            g = graphgen.symmetrize(g)
        order = rng.permutation(n).astype(np.int32)
        loff, src, dist = oracle.le_lists(g.n, g.out_off, g.out_adj, order)
        assert _le_rows(loff, src, dist, g.n) == _le_by_definition(g, order)


def test_le_lists_closed_forms():
    # undirected path in natural order: L(u) = 0, 1, ..., u at distances u, ..., 0
    n = 200
    g = graphgen.symmetrize(csr_of(n, [(i, i + 1) for i in range(n - 1)]))
    loff, src, dist = oracle.le_lists(n, g.out_off, g.out_adj, np.arange(n, dtype=np.int32))
    rows = _le_rows(loff, src, dist, n)
    for u in range(n):
        assert rows[u] == [(s, u - s) for s in range(u + 1)]
    # every list ends with the vertex itself at distance 0; the first vertex of
    # the order heads the list of everything it reaches
    h = graphgen.symmetrize(graphgen.torus(20, 20, 0.6, seed=3))
    order = np.random.default_rng(2).permutation(h.n).astype(np.int32)
    loff, src, dist = oracle.le_lists(h.n, h.out_off, h.out_adj, order)
    reach0 = set(oracle.reach_pairs(h.n, h.out_off, h.out_adj, np.zeros(h.n, np.int32), [order[0]])[:, 0].tolist())
    for u in range(h.n):
        assert src[loff[u + 1] - 1] == u and dist[loff[u + 1] - 1] == 0
        assert (src[loff[u]] == order[0]) == (u in reach0)
        assert np.all(np.diff(dist[loff[u]:loff[u + 1]]) < 0)
