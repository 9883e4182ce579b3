"""Schedule autotuner for batched SCC runs.

A batch of many graphs runs as one disjoint union (``scc_labels_batched``),
so one schedule -- the local-search budget tau (Section 3.2), the
prefix-doubling multiplier beta (Algorithm 1) and the faster multiplier
beta_fast used after latency-bound source batches -- serves every graph of
it.  None of them changes the labels, only rounds and work, and the best
values depend on the graphs (k-NN graphs and short-diameter graphs gain from
fast batch growth, long lattices lose) and on the batch's size: beta sets how
many source batches a run takes, log_beta(n), so a sample must keep the
scale of the whole batch.  The tuner times a few candidate schedules on a
sample of the batch (every k-th graph, k >= 2, from a seeded offset; by
default every second graph, a strict subset that keeps the batch's scale), on
the GPU, and returns the fastest as options for the whole batch.  It then
times the chosen schedule and the default one on the graphs it did not see,
so that the reported gain is measured out of sample.

All timing goes through the library's C ABI; this module only chooses
which options to pass.
"""
from __future__ import annotations

import time

import numpy as np

from . import _native

# candidate (tau, beta, beta_fast, policy) schedules, the defaults first;
# policy 1 lets the learned per-round policy pick the budget (tau is then its
# fallback), so the tuner also decides whether the policy is used
CANDIDATES = [(2048, 2.0, 4.0, 0), (2048, 2.0, 8.0, 0), (2048, 2.0, 24.0, 0), (4096, 2.0, 8.0, 0),
              (2048, 3.0, 8.0, 0), (4096, 2.0, 24.0, 0), (1024, 2.0, 16.0, 0), (2048, 2.0, 4.0, 1),
              (2048, 2.0, 24.0, 1)]


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


def _time_batch(vb, ab, arrs, o, repeats):
    import torch

    from . import scc_labels_batched
    ts = []
    for r in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        scc_labels_batched(vb, ab, *arrs, options=o)
        torch.cuda.synchronize()
        if r:  # the first call warms up (allocations)
            ts.append((time.perf_counter() - t0) * 1e3)
    return min(ts)


def split(vb, ab, sample_arcs: int | None = None, seed: int = 0):
    """Indices of the tuning sample and of the held-out graphs: every k-th
    graph from a seeded offset, k = max(2, total arcs // sample_arcs)."""
    vb = np.asarray(vb, np.int64)
    ab = np.asarray(ab, np.int64)
    G = len(vb) - 1
    total = int(ab[-1]) if G else 0
    if sample_arcs is None:
        sample_arcs = total // 2
    stride = max(2, int(total // max(sample_arcs, 1)))
    off = int(np.random.default_rng(seed).integers(0, stride)) if G else 0
    idx = list(range(off, G, stride))
    seen = set(idx)
    rest = [g for g in range(G) if g not in seen]
    return idx, rest


MARGIN = 0.03  # a candidate must beat the first (the library default) by this fraction on the sample


def choose(times, margin=MARGIN):
    """Index of the schedule to use: the fastest, unless it is not `margin`
    faster than the first (the default), which then stays."""
    best = min(range(len(times)), key=lambda i: times[i])
    return best if times[best] < times[0] * (1.0 - margin) else 0


def tune(vb, ab, out_off, out_adj, in_off, in_adj, sample_arcs: int | None = None, repeats: int = 1,
         candidates=CANDIDATES, base_options=None, verbose: bool = False, seed: int = 0, held_out: bool = True,
         margin: float = MARGIN):
    """Pick (tau, beta, beta_fast, policy) for a batch.  Returns (options, report):
    each candidate's best time on the sample, and (held_out) the chosen and
    the default schedule's times on the graphs outside the sample.  The first
    candidate stays unless another is faster on the sample by `margin`, so
    that timing noise between near-equal schedules does not pick the schedule."""
    from . import default_options
    vb = np.asarray(vb, np.int64)
    ab = np.asarray(ab, np.int64)
    arrays = (out_off, out_adj, in_off, in_adj)
    idx, rest = split(vb, ab, sample_arcs, seed)
    svb, sab, sarr = _subset(vb, ab, arrays, idx)
    report = []
    for cand in candidates:
        tau, beta, beta_fast = cand[:3]
        policy = cand[3] if len(cand) > 3 else 0
        o = default_options() if base_options is None else _copy(base_options)
        o.tau = tau
        o.beta = beta
        o.beta_fast = beta_fast
        o.policy = policy
        o.timing = 0
        ms = _time_batch(svb, sab, sarr, o, repeats)
        report.append({"tau": tau, "beta": beta, "beta_fast": beta_fast, "policy": policy, "sample_ms": ms})
        if verbose:
            print("[autotune] tau=%d beta=%.1f beta_fast=%.0f policy=%d sample %.2f ms" %
                  (tau, beta, beta_fast, policy, ms), flush=True)
    del sarr
    o = default_options() if base_options is None else _copy(base_options)
    if report:
        b = report[choose([r["sample_ms"] for r in report], margin)]
        o.tau, o.beta, o.beta_fast, o.policy = b["tau"], b["beta"], b["beta_fast"], b["policy"]
    rep = {"sample_graphs": len(idx), "sample_arcs": int(sab[-1]) if len(idx) else 0,
           "held_out_graphs": len(rest), "candidates": report}
    if held_out and rest:
        hvb, hab, harr = _subset(vb, ab, arrays, rest)
        d = default_options() if base_options is None else _copy(base_options)
        d.timing = 0
        d.policy = 0
        o.timing = 0
        rep["held_out_tuned_ms"] = _time_batch(hvb, hab, harr, o, repeats)
        rep["held_out_default_ms"] = _time_batch(hvb, hab, harr, d, repeats)
        rep["held_out_arcs"] = int(hab[-1])
        del harr
    return o, rep


def _copy(o):
    c = _native.Options()
    for f, _ in o._fields_:
        setattr(c, f, getattr(o, f))
    return c
