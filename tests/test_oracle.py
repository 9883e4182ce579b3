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
