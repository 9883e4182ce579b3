"""The allocation-free entry point (scc_labels_static) against scc_labels.

Both are called through the C ABI on the same graphs; labels must agree bit
for bit.  Two calls in a row, the second on a smaller graph, check that the
shared static scratch carries nothing from one call into the next.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _pair(gpu, g, opts=None):
    import torch
    dg = gpu.to_device(g)
    want = gpu.scc_labels(dg, opts).cpu().numpy()
    out = torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda")
    got, st = gpu.scc_labels_static(dg, out, opts, return_stats=True)
    got = got.cpu().numpy()
    assert np.array_equal(got, want), "static labels differ from scc_labels on %s" % g.name
    assert st["n_scc"] == len(np.unique(want))
    return got


def test_static_matches_scc_labels_twice_second_smaller(gpu):
    big = graphgen.torus(300, 400, 0.5, seed=501)
    small = graphgen.rmat(12, 8, seed=502)
    say("static big", big.n, big.m)
    a = _pair(gpu, big)
    say("static small", small.n, small.m)
    b = _pair(gpu, small)
    assert np.array_equal(a, oracle.scc_graph(big))
    assert np.array_equal(b, oracle.scc_graph(small))


def test_static_config0_full_size_and_tiny(gpu):
    g = graphgen.config(0)
    say("static config0", g.n, g.m)
    _pair(gpu, g)
    t = graphgen.random_digraph(50, 1.5, seed=503)
    say("static tiny", t.n, t.m)
    _pair(gpu, t)
    e = graphgen.from_arcs(1, [], [])
    _pair(gpu, e)


def test_static_options_and_rejections(gpu):
    import torch
    g = graphgen.knn(30000, 3, 5, 0.01, seed=504)
    say("static knn options")
    _pair(gpu, g, gpu.default_options(tau=1, beta=1.5))
    _pair(gpu, g, gpu.default_options(dense=1))
    dg = gpu.to_device(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.SccError) as e:
        gpu.scc_labels_static(dg, out, gpu.default_options(timing=1))
    assert e.value.code == -1
    # a graph beyond the static scratch is refused before any work
    n = 3_000_000
    z = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    a = torch.zeros(1, dtype=torch.int32, device="cuda")
    huge = gpu.DeviceGraph(n, 0, z, a, z, a)
    with pytest.raises(gpu.SccError) as e:
        gpu.scc_labels_static(huge, torch.empty(n, dtype=torch.int32, device="cuda"))
    assert e.value.code == -4
    # the context still works, on both entry points
    _pair(gpu, graphgen.torus(50, 50, 0.6, seed=505))
