"""Batched execution (many graphs as one disjoint union) against the oracle,
with the schedule autotuner's choice, and the per-graph loop it replaces."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def test_autotuned_batch_matches_oracle_and_per_graph_calls(gpu):
    import torch
    from paper_2303_04934_amd import autotune
    graphs = graphgen.batched(300, seed=4242, lo_exp=2.0, hi_exp=4.0)
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    print("[case] autotuned batch", len(graphs), "graphs", int(vb[-1]), "vertices", int(ab[-1]), "arcs", flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    arrs = (t(oo), t(oa), t(io), t(ia))
    opts, rep = autotune.tune(vb, ab, *arrs, sample_arcs=200_000, repeats=1)
    assert (opts.tau, opts.beta) in [(c[0], pytest.approx(c[1])) for c in autotune.CANDIDATES]
    assert len(rep["candidates"]) == len(autotune.CANDIDATES) and rep["sample_graphs"] > 0
    # the sample is a strict subset; the chosen schedule was also timed on the rest
    assert 0 < rep["held_out_graphs"] < len(graphs) and rep["sample_graphs"] + rep["held_out_graphs"] == len(graphs)
    assert rep["held_out_tuned_ms"] > 0 and rep["held_out_default_ms"] > 0
    got = gpu.scc_labels_batched(vb, ab, *arrs, options=opts).cpu().numpy()
    for g, gr in enumerate(graphs):
        assert np.array_equal(got[vb[g]:vb[g + 1]], oracle.scc_graph(gr)), "graph %d" % g
    # the same graphs one call each (device views of the batch arrays)
    for g in range(0, len(graphs), 37):
        n, lo = int(vb[g + 1] - vb[g]), int(vb[g]) + g
        dg = gpu.DeviceGraph(n, int(ab[g + 1] - ab[g]), arrs[0][lo:lo + n + 1], arrs[1][int(ab[g]):int(ab[g + 1])],
                             arrs[2][lo:lo + n + 1], arrs[3][int(ab[g]):int(ab[g + 1])])
        assert np.array_equal(gpu.scc_labels(dg).cpu().numpy(), got[vb[g]:vb[g + 1]])


def test_batch_split_into_several_unions(gpu):
    # a batch whose arcs exceed the union limit runs as several disjoint
    # unions (the path the full 4096-graph batch takes at 2^31 arcs); here the
    # limit is lowered so that a small batch splits into many unions, one of
    # them a single graph larger than the limit, run one after another, two
    # or four at a time (more unions than streams: each worker runs several)
    import torch
    graphs = graphgen.batched(60, seed=4343, lo_exp=2.0, hi_exp=3.6)
    graphs.insert(17, graphgen.torus(250, 260, 0.6, seed=4344))
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    total = int(ab[-1])
    limit = max(total // 7, 1000)
    biggest = int(np.max(np.diff(ab)))
    assert biggest > limit and total > 3 * limit
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    arrs = (t(oo), t(oa), t(io), t(ia))
    want = [oracle.scc_graph(gr) for gr in graphs]
    for streams in (1, 2, 4):
        print("[case] batch split", len(graphs), "graphs", total, "arcs, limit", limit, "streams", streams,
              flush=True)
        got, st = gpu.scc_labels_batched(vb, ab, *arrs,
                                         options=gpu.default_options(union_arcs_max=limit, union_streams=streams),
                                         return_stats=True)
        got = got.cpu().numpy()
        for g in range(len(graphs)):
            assert np.array_equal(got[vb[g]:vb[g + 1]], want[g]), "graph %d streams %d" % (g, streams)
        assert st["n_scc"] == sum(len(np.unique(w)) for w in want)


def test_concurrent_unions_match_oracle(gpu):
    # unions on concurrent streams (worker contexts driven by host threads):
    # every stream count gives the oracle's labels, on repeated calls (the
    # workers and their buffers are reused), with kernel timing on, and with
    # the learned policy (its weights copied to the workers)
    import os
    import torch
    graphs = graphgen.batched(160, seed=4646, lo_exp=2.0, hi_exp=3.8)
    graphs.insert(40, graphgen.torus(200, 180, 0.5, seed=4647))
    graphs.insert(110, graphgen.grid(150, 220, 0.5, seed=4648))
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    arrs = (t(oo), t(oa), t(io), t(ia))
    want = [oracle.scc_graph(gr) for gr in graphs]
    gpu.policy_load(np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                         "paper_2303_04934_amd", "policy_weights.npy")))
    cases = [dict(union_streams=s) for s in (0, 1, 2, 3, 5)]
    cases += [dict(union_streams=2, timing=0x7f), dict(union_streams=3, policy=1), dict(union_streams=2, first_slot=0)]
    for kw in cases:
        for rep in range(2):
            print("[case] concurrent unions %s rep %d" % (kw, rep), flush=True)
            got, st = gpu.scc_labels_batched(vb, ab, *arrs, options=gpu.default_options(**kw), return_stats=True)
            got = got.cpu().numpy()
            for g in range(len(graphs)):
                assert np.array_equal(got[vb[g]:vb[g + 1]], want[g]), "graph %d %s" % (g, kw)
            assert st["n_scc"] == sum(len(np.unique(w)) for w in want)
            if kw.get("timing"):  # every frontier kernel timed (a bit per kernel)
                assert st["launches_kernel"][1] > 0 and st["ms_kernel"][1] > 0


def test_batch_with_graph_rounds_and_learned_policy(gpu):
    import os
    import torch
    graphs = graphgen.batched(120, seed=4545, lo_exp=2.0, hi_exp=3.8)
    vb, ab, oo, oa, io, ia = graphgen.concat(graphs)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    arrs = (t(oo), t(oa), t(io), t(ia))
    gpu.policy_load(np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                         "paper_2303_04934_amd", "policy_weights.npy")))
    for opts in (gpu.default_options(graph_rounds=1), gpu.default_options(policy=1)):
        for rep in range(2):
            print("[case] batch graph_rounds=%d policy=%d rep %d" % (opts.graph_rounds, opts.policy, rep), flush=True)
            got = gpu.scc_labels_batched(vb, ab, *arrs, options=opts).cpu().numpy()
            for g, gr in enumerate(graphs):
                assert np.array_equal(got[vb[g]:vb[g + 1]], oracle.scc_graph(gr)), "graph %d" % g
