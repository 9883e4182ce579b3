"""GPU parity of connected components (LDD-UF-JTB, Algorithm 4) against the
oracle's sequential union-find: labels (smallest vertex id per component)
must match bit for bit, on symmetric graphs (connected components) and on
digraphs (weakly connected components), for every schedule."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def check_cc(scc, g, opts=None, name=""):
    say("scc_cc", name or g.name, "n=%d m=%d" % (g.n, g.m))
    dg = scc.to_device(g)
    got, st = scc.scc_cc(dg, opts, return_stats=True)
    got = got.cpu().numpy()
    want = oracle.wcc_labels(g.n, g.out_off, g.out_adj)
    assert np.array_equal(got, want), "component labels differ on %s (first bad vertex %s)" % (
        name or g.name, np.nonzero(got != want)[0][:5])
    assert st["n_scc"] == len(np.unique(want))
    return st


@pytest.mark.parametrize("which", ["rmat13", "knn30k", "torus80", "sqr2_60", "er_sparse", "path"])
def test_cc_symmetric_families(gpu, which):
    g = {"rmat13": lambda: graphgen.rmat(13, 8, seed=71),
         "knn30k": lambda: graphgen.knn(30000, 3, 5, 0.01, seed=72),
         "torus80": lambda: graphgen.torus(80, 90, 0.3, seed=73),
         "sqr2_60": lambda: graphgen.lattice_oriented(60, 70, 1, seed=74),
         "er_sparse": lambda: graphgen.random_digraph(20000, 0.6, seed=75),
         "path": lambda: graphgen.from_arcs(30000, np.arange(29999), np.arange(1, 30000))}[which]()
    check_cc(gpu, graphgen.symmetrize(g), name=which + "_sym")


def test_cc_directed_inputs_give_weak_components(gpu):
    for g in (graphgen.rmat(12, 4, seed=76), graphgen.grid(70, 80, 0.3, seed=77),
              graphgen.random_digraph(5000, 0.9, seed=78)):
        check_cc(gpu, g, name=g.name + " (directed)")


@pytest.mark.parametrize("opt", [dict(), dict(tau=1), dict(tau=64), dict(tau=65536), dict(ldd_beta=1.05),
                                 dict(ldd_beta=2.0), dict(ldd_beta=64.0), dict(seed=99), dict(vgc_measure=1),
                                 dict(lambda_log2=6, sigma=1, kappa=0)])
def test_cc_schedule_invariance(gpu, opt):
    g = graphgen.symmetrize(graphgen.torus(120, 130, 0.35, seed=79))
    check_cc(gpu, g, gpu.default_options(**opt), name="torus120x130 %s" % opt)


def test_cc_degenerate(gpu):
    check_cc(gpu, graphgen.from_arcs(1, [], []), name="n1")
    check_cc(gpu, graphgen.from_arcs(7, [], []), name="n7 no arcs")
    check_cc(gpu, graphgen.from_arcs(5, [0, 1, 2, 3, 4], [0, 1, 2, 3, 4]), name="self loops")
    star = graphgen.symmetrize(graphgen.from_arcs(50000, np.zeros(49999, np.int64), np.arange(1, 50000)))
    check_cc(gpu, star, name="star50000")
    import torch
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert gpu.scc_cc(gpu.DeviceGraph(0, 0, z, e, z, e)).numel() == 0


@pytest.mark.parametrize("cfg,shrink", [(1, 2), (2, 0), (7, 0)], ids=["rmat_s22_ef16_sym", "knn_10M_k5_sym",
                                                                       "sqr2_10000_sym"])
def test_cc_full_size(gpu, cfg, shrink):
    g = graphgen.symmetrize(graphgen.config(cfg, shrink=shrink))
    st = check_cc(gpu, g, name="%s full size" % g.name)
    assert st["rounds_first"] > 0
