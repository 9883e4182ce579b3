"""GPU parity at the full sizes of the benchmark workloads.

Every SCC label of the HIP path is compared with the sequential oracle's, bit
for bit, with the default options (the configuration bench.py times).  The
multi-source reach path is checked at full size on a sample of sources, each
source's reach set recomputed by the oracle's BFS.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [1, 2, 3], ids=["rmat_s24_ef16", "knn_10M_k5", "grid10000_p0.5"])
def test_full_size_labels_match_oracle(gpu, cfg):
    g = graphgen.config(cfg)
    print("[case] full-size labels", g.name, "n=%d m=%d" % (g.n, g.m), flush=True)
    dg = gpu.to_device(g)
    got, st = gpu.scc_labels(dg, gpu.default_options(timing=1), return_stats=True)
    got = got.cpu().numpy()
    want = oracle.scc_graph(g)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "labels differ at %d vertices, first %s" % (bad.size, bad[:5])
    assert st["n_scc"] == len(np.unique(want))
    assert st["batches"] > 1


@pytest.mark.parametrize("cfg", [5, 6, 7, 8], ids=["sqr_10000", "rec_1000x10000", "sqr2_10000", "rec2_1000x10000"])
def test_paper_lattices_full_size(gpu, cfg):
    # the paper's own lattices (Section 6, Table 3) at full size, bit-exact
    g = graphgen.config(cfg)
    print("[case] full-size paper lattice", g.name, "n=%d m=%d" % (g.n, g.m), flush=True)
    dg = gpu.to_device(g)
    got, st = gpu.scc_labels(dg, return_stats=True)
    got = got.cpu().numpy()
    want = oracle.scc_graph(g)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "labels differ at %d vertices, first %s" % (bad.size, bad[:5])
    sizes = np.bincount(want)
    print("[case] %s: #SCC %d, largest %d (%.2f%%)" % (g.name, st["n_scc"], sizes.max(), 100.0 * sizes.max() / g.n),
          flush=True)
    assert st["n_scc"] == int(np.count_nonzero(sizes))


def test_full_size_multi_source_reach(gpu):
    g = graphgen.config(2)
    rng = np.random.default_rng(2024)
    srcs = [int(x) for x in rng.choice(g.n, size=6, replace=False)]
    lab = np.zeros(g.n, np.int32)
    dg = gpu.to_device(g)
    for d in (0, 1):
        print("[case] full-size reach", g.name, "direction", d, srcs, flush=True)
        got = gpu.scc_reach(dg, srcs, lab, direction=d).cpu().numpy()
        off, adj = (g.out_off, g.out_adj) if d == 0 else (g.in_off, g.in_adj)
        want = oracle.reach_pairs(g.n, off, adj, lab, srcs)
        assert np.array_equal(got, want)  # both sorted by (source index, vertex)
