"""Input generators: determinism, structure and exactness (CPU only)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen


def _csr_ok(g):
    assert g.out_off[0] == 0 and g.out_off[-1] == g.m and np.all(np.diff(g.out_off) >= 0)
    assert g.in_off[0] == 0 and g.in_off[-1] == g.m and np.all(np.diff(g.in_off) >= 0)
    if g.m:
        assert g.out_adj.min() >= 0 and g.out_adj.max() < g.n
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    isrc = np.repeat(np.arange(g.n), np.diff(g.in_off))
    a = np.sort(src.astype(np.int64) * g.n + g.out_adj)
    b = np.sort(g.in_adj.astype(np.int64) * g.n + isrc)
    assert np.array_equal(a, b), "transpose is not the same arc multiset"
    return src


def test_lattice_matches_definition():
    rows, cols, p, seed = 7, 9, 0.5, 42
    for wrap in (True, False):
        g = graphgen.lattice(rows, cols, p, seed, wrap)
        src = _csr_ok(g)
        want = set()
        for u in range(rows * cols):
            r, c = divmod(u, cols)
            for d, (dr, dc) in enumerate([(0, 1), (0, -1), (1, 0), (-1, 0)]):
                rr, cc = r + dr, c + dc
                if wrap:
                    rr, cc = rr % rows, cc % cols
                elif not (0 <= rr < rows and 0 <= cc < cols):
                    continue
                if graphgen.unif(seed, 0, 4 * u + d) < p:
                    want.add((u, rr * cols + cc))
        assert set(zip(src.tolist(), g.out_adj.tolist())) == want


def test_rmat_structure():
    g = graphgen.rmat(12, 16, seed=5)
    src = _csr_ok(g)
    assert g.n == 4096 and 0.8 * 16 * 4096 < g.m <= 16 * 4096
    assert not np.any(src == g.out_adj), "self loop"
    key = src.astype(np.int64) * g.n + g.out_adj
    assert len(np.unique(key)) == g.m, "duplicate arc"
    deg = np.diff(g.out_off)
    assert deg.max() > 20 * deg.mean(), "R-MAT should be skewed"


def test_knn_exact_against_bruteforce():
    g, pts = graphgen.knn(3000, 3, 5, 0.01, seed=8, return_points=True)
    _csr_ok(g)
    assert np.all(np.diff(g.out_off) == 5)
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    for i in range(0, 3000, 37):
        order = np.lexsort((np.arange(3000), d2[i]))[:5]
        assert np.array_equal(np.sort(order), g.out_adj[g.out_off[i]:g.out_off[i + 1]])


def test_thread_count_independence(tmp_path):
    code = ("import graphgen, hashlib, numpy as np\n"
            "h = hashlib.sha256()\n"
            "for g in (graphgen.rmat(12, 8, seed=3), graphgen.knn(5000, 5, 5, 0.01, seed=3),"
            " graphgen.torus(50, 60, 0.5, seed=3)):\n"
            "    for a in (g.out_off, g.out_adj, g.in_off, g.in_adj): h.update(a.tobytes())\n"
            "print(h.hexdigest())\n")
    outs = []
    for t in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env, cwd=root).strip())
    assert outs[0] == outs[1]


def test_config_small_shapes():
    g0 = graphgen.config(0, shrink=6)
    _csr_ok(g0)
    assert abs(g0.m - 2 * g0.n) < 0.05 * g0.n
    g3 = graphgen.config(3, shrink=12)
    _csr_ok(g3)
    spec = graphgen.batched_spec(64)
    assert all(1000 <= n <= 1_000_000 for _, n, _ in spec)
    assert {f for f, _, _ in spec} == {0, 1, 2}


def test_from_arcs_rejects_bad_input():
    with pytest.raises(ValueError):
        graphgen.from_arcs(3, [0, 5], [1, 2])
    g = graphgen.from_arcs(3, [0, 0, 1], [1, 1, 1])
    assert g.m == 3  # duplicates and self loops kept unless dedup


def test_oriented_lattices_match_definition():
    # the paper's lattices (Section 6) recomputed arc by arc from the draws
    rows, cols, seed = 6, 8, 77
    n = rows * cols
    for mode in (0, 1):
        g = graphgen.lattice_oriented(rows, cols, mode, seed)
        src = _csr_ok(g)
        want = set()
        for u in range(n):
            r, c = divmod(u, cols)
            east, south = r * cols + (c + 1) % cols, ((r + 1) % rows) * cols + c
            if mode == 0:
                nbrs = [east, r * cols + (c - 1) % cols, south, ((r - 1) % rows) * cols + c]
                for d, v in enumerate(nbrs):  # u's own draw for each adjacent vertex
                    if graphgen.unif(seed, 2, 4 * u + d) < 0.5:
                        want.add((u, v))
                    else:
                        want.add((v, u))
            else:
                for j, v in enumerate((east, south)):  # u owns its east and south edges
                    if graphgen.unif(seed, 3, 4 * u + 2 * j) < 0.3:
                        want.add((u, v))
                    if graphgen.unif(seed, 3, 4 * u + 2 * j + 1) < 0.3:
                        want.add((v, u))
        got = set(zip(src.tolist(), g.out_adj.tolist()))
        assert got == want, mode
        assert len(got) == g.m  # duplicates removed


def test_oriented_lattice_arc_density():
    # Table 3: SQR has 300M arcs on 2e8 edges (1.5 per edge), SQR' 120M (0.6)
    for mode, per_edge in ((0, 1.5), (1, 0.6)):
        g = graphgen.lattice_oriented(300, 400, mode, 5)
        assert abs(g.m / (2 * g.n) - per_edge) < 0.01
        src = np.repeat(np.arange(g.n), np.diff(g.out_off))
        assert not np.any(src == g.out_adj)
    # mode 0 orients every edge at least one way
    g = graphgen.lattice_oriented(50, 60, 0, 6)
    und = set()
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    for u, v in zip(src.tolist(), g.out_adj.tolist()):
        und.add((min(u, v), max(u, v)))
    assert len(und) == 2 * g.n
