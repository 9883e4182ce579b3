"""Schedule autotuner for batched SCC runs.

A batch of many graphs runs as one disjoint union (``scc_labels_batched``),
so one schedule -- the local-search budget tau (Section 3.2), the
prefix-doubling multiplier beta (Algorithm 1) and the faster multiplier
beta_fast used after latency-bound source batches -- serves every graph of
it.  None of them changes the labels, only rounds and work, and the best
values depend on the graphs (k-NN graphs and short-diameter graphs gain from
fast batch growth, long lattices lose) and on the batch's size: beta sets how
many source batches a run takes, log_beta(n), so a sample must keep the
scale of the whole batch.  The tuner times a few candidate schedules on a sample of the
batch (every k-th graph; by default every second one), on the GPU, and
returns the fastest as options for the whole batch.

All timing goes through the library's C ABI; this module only chooses
which options to pass.
"""
from __future__ import annotations

import time

import numpy as np

from . import _native

# candidate (tau, beta, beta_fast) schedules: the defaults first
CANDIDATES = [(2048, 2.0, 8.0), (2048, 2.0, 24.0), (4096, 2.0, 8.0), (2048, 3.0, 8.0), (4096, 2.0, 24.0),
              (1024, 2.0, 16.0)]


def _subset(vb, ab, arrays, idx):
    """Concatenated device arrays and bases of the graphs in idx (views copied once)."""
    import torch
    oo, oa, io, ia = arrays
    vb2 = np.zeros(len(idx) + 1, np.int64)
    ab2 = np.zeros(len(idx) + 1, np.int64)
    po, pa, pi, pia = [], [], [], []
    for j, g in enumerate(idx):
        n = int(vb[g + 1] - vb[g])
        m = int(ab[g + 1] - ab[g])
        vb2[j + 1] = vb2[j] + n
        ab2[j + 1] = ab2[j] + m
        lo = int(vb[g]) + g
        po.append(oo[lo:lo + n + 1])
        pi.append(io[lo:lo + n + 1])
        pa.append(oa[int(ab[g]):int(ab[g]) + m])
        pia.append(ia[int(ab[g]):int(ab[g]) + m])
    cat = lambda xs: torch.cat(xs) if xs else torch.zeros(0, dtype=torch.int32, device=oo.device)
    return vb2, ab2, (cat(po), cat(pa), cat(pi), cat(pia))


def tune(vb, ab, out_off, out_adj, in_off, in_adj, sample_arcs: int | None = None, repeats: int = 1,
         candidates=CANDIDATES, base_options=None, verbose: bool = False):
    """Pick (tau, beta, beta_fast) for a batch.  Returns (options, report)
    where report lists each candidate's best sample time in ms."""
    import torch

    from . import default_options, scc_labels_batched
    vb = np.asarray(vb, np.int64)
    ab = np.asarray(ab, np.int64)
    G = len(vb) - 1
    total = int(ab[-1])
    if sample_arcs is None:
        sample_arcs = (total + 1) // 2
    stride = max(1, int(total // max(sample_arcs, 1)))
    idx = list(range(0, G, stride)) if G else []
    svb, sab, sarr = _subset(vb, ab, (out_off, out_adj, in_off, in_adj), idx)
    report = []
    best = None
    for tau, beta, beta_fast in candidates:
        o = default_options() if base_options is None else _copy(base_options)
        o.tau = tau
        o.beta = beta
        o.beta_fast = beta_fast
        o.timing = 0
        ts = []
        for r in range(repeats + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            scc_labels_batched(svb, sab, *sarr, options=o)
            torch.cuda.synchronize()
            if r:  # the first call warms up (allocations)
                ts.append((time.perf_counter() - t0) * 1e3)
        ms = min(ts)
        report.append({"tau": tau, "beta": beta, "beta_fast": beta_fast, "sample_ms": ms})
        if verbose:
            print("[autotune] tau=%d beta=%.1f beta_fast=%.0f sample %.2f ms" % (tau, beta, beta_fast, ms),
                  flush=True)
        if best is None or ms < best[0]:
            best = (ms, tau, beta, beta_fast)
    o = default_options() if base_options is None else _copy(base_options)
    if best is not None:
        o.tau, o.beta, o.beta_fast = best[1], best[2], best[3]
    return o, {"sample_graphs": len(idx), "sample_arcs": int(sab[-1]) if len(idx) else 0, "candidates": report}


def _copy(o):
    c = _native.Options()
    for f, _ in o._fields_:
        setattr(c, f, getattr(o, f))
    return c
