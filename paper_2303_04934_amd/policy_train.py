"""Learned round policy: trace collection (GPU) and offline training (NumPy).

The policy is a float32 MLP 5 -> 32 -> 32 -> 8 (ReLU) that the library runs
on the device before every search round (``options.policy = 1``).  Its inputs
are the round features of ``scc_trace_read`` (frontier size, frontier degree
sum, visited fraction, round index, deepest local search of the previous
round); output 2c + m scores budget class c (64 * 4^c arcs) with frontier mode
m (0 sparse, 1 dense).  The library takes the best allowed output.

Training data are per-round traces of runs that draw a random budget class
every round (``options.policy = 2``) on training graphs whose seeds (>= 10^6)
are disjoint from the benchmark inputs.  Each row gives the taken action and
the round's outcome; the regression target is the round's progress rate
log((entries claimed + 1) / (round ms + launch overhead)).  Only the taken
action's output is trained (dense rounds train all four dense outputs, whose
budget does not matter).  The policy only chooses schedules: the SCC labels
do not depend on it.

    python -m paper_2303_04934_amd.policy_train collect --out traces.npy   # on a GPU
    python -m paper_2303_04934_amd.policy_train fit traces.npy --out policy_weights.npy
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "policy_weights.npy")
N_IN, HID, N_OUT = 5, 32, 8
ROUND_OVERHEAD_MS = 0.03  # launch + check cost a round adds beyond its kernels


def n_params():
    return HID * N_IN + HID + HID * HID + HID + N_OUT * HID + N_OUT


def unpack(w):
    o = 0
    out = []
    for r, c in ((HID, N_IN), (1, HID), (HID, HID), (1, HID), (N_OUT, HID), (1, N_OUT)):
        out.append(w[o:o + r * c].reshape(r, c) if r > 1 else w[o:o + c])
        o += r * c
    return out


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3]).astype(np.float32)


def forward(w, x):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    h1 = np.maximum(x @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    return h2 @ W3.T + b3, (h1, h2)


def dataset(rows):
    """(features, action mask, target) from trace rows."""
    rows = np.asarray(rows, np.float64)
    x = rows[:, 1:6].astype(np.float32)
    kind, tau, ms, claims = rows[:, 0], rows[:, 6], rows[:, 7], rows[:, 8]
    y = np.log((claims + 1.0) / (ms + ROUND_OVERHEAD_MS)).astype(np.float32)
    mask = np.zeros((len(rows), N_OUT), np.float32)
    cls = np.clip(np.round(np.log(np.maximum(tau, 64) / 64.0) / np.log(4.0)), 0, 3).astype(int)
    dense = kind == 1
    mask[~dense, 2 * cls[~dense]] = 1.0
    mask[dense, 1::2] = 1.0
    return x, mask, y


def fit(rows, steps=4000, lr=3e-3, seed=0, verbose=True):
    """Masked-MSE regression of the taken actions' rates; Adam, full batch."""
    x, mask, y = dataset(rows)
    rng = np.random.default_rng(seed)
    p = [rng.standard_normal((HID, N_IN)) * np.sqrt(2 / N_IN), np.zeros(HID),
         rng.standard_normal((HID, HID)) * np.sqrt(2 / HID), np.zeros(HID),
         rng.standard_normal((N_OUT, HID)) * np.sqrt(1 / HID), np.full(N_OUT, float(y.mean()))]
    p = [a.astype(np.float64) for a in p]
    m = [np.zeros_like(a) for a in p]
    v = [np.zeros_like(a) for a in p]
    X = x.astype(np.float64)
    Y = y.astype(np.float64)[:, None]
    M = mask.astype(np.float64)
    cnt = max(M.sum(), 1.0)
    for it in range(1, steps + 1):
        h1p = X @ p[0].T + p[1]
        h1 = np.maximum(h1p, 0)
        h2p = h1 @ p[2].T + p[3]
        h2 = np.maximum(h2p, 0)
        out = h2 @ p[4].T + p[5]
        err = (out - Y) * M
        loss = (err ** 2).sum() / cnt
        g_out = 2 * err / cnt
        g = [None] * 6
        g[4] = g_out.T @ h2
        g[5] = g_out.sum(0)
        g_h2 = (g_out @ p[4]) * (h2p > 0)
        g[2] = g_h2.T @ h1
        g[3] = g_h2.sum(0)
        g_h1 = (g_h2 @ p[2]) * (h1p > 0)
        g[0] = g_h1.T @ X
        g[1] = g_h1.sum(0)
        for i in range(6):
            m[i] = 0.9 * m[i] + 0.1 * g[i]
            v[i] = 0.999 * v[i] + 0.001 * g[i] ** 2
            mh = m[i] / (1 - 0.9 ** it)
            vh = v[i] / (1 - 0.999 ** it)
            p[i] -= lr * mh / (np.sqrt(vh) + 1e-8)
        if verbose and (it % 1000 == 0 or it == 1):
            print("step %d loss %.4f" % (it, loss), flush=True)
    return pack(*p)


def training_graphs():
    """Small graphs of every family with seeds disjoint from the benchmark inputs."""
    import graphgen
    out = []
    for i in range(2):
        s = 1_000_000 + 17 * i
        out.append(graphgen.torus(400 + 100 * i, 500, 0.5, seed=s))
        out.append(graphgen.grid(800 + 200 * i, 800, 0.5, seed=s + 1))
        out.append(graphgen.knn(400_000 + 200_000 * i, 40 + 20 * i, 5, 0.01, seed=s + 2))
        out.append(graphgen.rmat(17 + i, 16, seed=s + 3))
    return out


def collect(runs_per_graph=3, verbose=True):
    """Exploration traces (random budget class per round) on the training graphs."""
    import paper_2303_04934_amd as scc
    rows = []
    for gi, g in enumerate(training_graphs()):
        dg = scc.to_device(g)
        for r in range(runs_per_graph):
            o = scc.default_options(policy=2, trace=1, seed=1_000_003 + 31 * gi + r, validate=0)
            scc.scc_labels(dg, o)
            t = scc.trace_read()
            rows.append(t)
            if verbose:
                print("[collect] %s run %d: %d rows" % (g.name, r, len(t)), flush=True)
    return np.concatenate(rows) if rows else np.zeros((0, 12), np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--runs", type=int, default=3)
    f = sub.add_parser("fit")
    f.add_argument("traces", nargs="+")
    f.add_argument("--out", default=WEIGHTS)
    f.add_argument("--steps", type=int, default=4000)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        rows = collect(a.runs)
        np.save(a.out, rows)
        print("saved %d rows to %s" % (len(rows), a.out))
    else:
        rows = np.concatenate([np.load(p) for p in a.traces])
        w = fit(rows, steps=a.steps)
        assert w.size == n_params()
        np.save(a.out, w)
        print("saved %d weights to %s" % (w.size, a.out))


if __name__ == "__main__":
    sys.exit(main())
