"""Sequential CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links, loads
or calls it, and it shares no code with the GPU path (the two only share the
seeded input generators in ``graphgen``).

Functions (plain definitions, see ``oracle.c`` for the citations):

* :func:`scc_labels`  -- Tarjan's SCC, canonical label = min vertex id per SCC;
* :func:`reach_pairs` -- per-source BFS reach restricted to label-equal arcs;
* :func:`check_partition` -- certificate (mutual reachability inside every
  class, acyclic class graph, label = class minimum);
* :func:`wcc_labels` -- weakly connected components (connected components of
  a symmetric digraph, Algorithm 4's output), canonical min id;
* :func:`le_lists` -- least-element lists for a given vertex order
  (Section 5.2), as CSR (offsets, sources, distances);
* :func:`bfs_depths` -- per-source BFS depth of the same restricted reach
  (the number of frontier rounds of Algorithm 2 is this depth plus one);
* :func:`hashbag_sim` -- a sequential model of the parallel hash bag
  (Section 3.3: doubling chunks, sampled load estimate, chunk moves, linear
  probing, ExtractAll over the used prefix), with the statistics Theorem 1
  bounds (load of a chunk when it is left, used prefix);
* :func:`hashbag_model` -- ExtractAll's output per round as the model
  produces it (sorted): the multiset inserted since the last extract;
* :func:`policy_forward` -- float32 forward pass of the round-policy MLP.

The C part is compiled with gcc (``build``); the MLP forward is numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.or_tarjan.argtypes = [i64, vp, vp, vp]
        lib.or_reach_pairs.argtypes = [i64, vp, vp, vp, i64, vp, vp, i64, ctypes.POINTER(i64)]
        lib.or_check_partition.argtypes = [i64, vp, vp, vp, vp, vp, ctypes.POINTER(i64)]
        lib.or_bfs_depths.argtypes = [i64, vp, vp, vp, i64, vp, vp]
        lib.or_wcc.argtypes = [i64, vp, vp, vp]
        lib.or_le_lists.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        lib.or_hashbag_sim.argtypes = [i64, vp, i64, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_uint64, vp, vp, vp, vp, vp, i64,
                                       ctypes.POINTER(i64)]
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def scc_labels(n: int, off, adj) -> np.ndarray:
    """labels[v] = minimum vertex id of v's strongly connected component."""
    off, adj = _i32(off), _i32(adj)
    out = np.empty(max(n, 1), np.int32)
    rc = _load().or_tarjan(n, off.ctypes.data, adj.ctypes.data if len(adj) else None, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("or_tarjan failed: %d" % rc)
    return out[:n]


def scc_graph(g) -> np.ndarray:
    return scc_labels(g.n, g.out_off, g.out_adj)


def reach_pairs(n: int, off, adj, labels, sources) -> np.ndarray:
    """Sorted (vertex, source_index) pairs, shape (count, 2), of the
    label-restricted reach from each source (arcs (u,w) need labels[u]==labels[w]>=0)."""
    off, adj, labels, sources = _i32(off), _i32(adj), _i32(labels), _i32(sources)
    lib = _load()
    cnt = ctypes.c_int64(0)
    cap = max(16, 4 * len(sources))
    while True:
        pairs = np.empty(2 * cap, np.int32)
        rc = lib.or_reach_pairs(n, off.ctypes.data, adj.ctypes.data if len(adj) else None, labels.ctypes.data,
                                len(sources), sources.ctypes.data if len(sources) else None, pairs.ctypes.data,
                                cap, ctypes.byref(cnt))
        if rc == -3:
            cap = int(cnt.value)
            continue
        if rc != 0:
            raise ValueError("or_reach_pairs rejected its input: %d" % rc)
        return pairs[: 2 * cnt.value].reshape(-1, 2)


def wcc_labels(n: int, off, adj) -> np.ndarray:
    """labels[v] = smallest vertex id of v's weakly connected component."""
    off, adj = _i32(off), _i32(adj)
    out = np.empty(max(n, 1), np.int32)
    rc = _load().or_wcc(n, off.ctypes.data, adj.ctypes.data if len(adj) else None, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("or_wcc failed: %d" % rc)
    return out[:n]


def le_lists(n: int, off, adj, order):
    """LE-lists for the vertex order ``order`` (order[i] = vertex at position
    i): (loff int64[n+1], src int32[count], dist int32[count]); vertex u's
    entries sit at [loff[u], loff[u+1]) in order of the sources' positions."""
    off, adj, order = _i32(off), _i32(adj), _i32(order)
    loff = np.zeros(n + 1, np.int64)
    cnt = ctypes.c_int64(0)
    cap = max(16, 8 * n)
    while True:
        src = np.empty(cap, np.int32)
        dist = np.empty(cap, np.int32)
        rc = _load().or_le_lists(n, off.ctypes.data, adj.ctypes.data if len(adj) else None,
                                 order.ctypes.data if n else None, loff.ctypes.data, src.ctypes.data,
                                 dist.ctypes.data, cap, ctypes.byref(cnt))
        if rc == -3:
            cap = int(cnt.value)
            continue
        if rc != 0:
            raise ValueError("or_le_lists failed: %d" % rc)
        k = int(cnt.value)
        return loff, src[:k].copy(), dist[:k].copy()


def check_partition(g, labels):
    """(code, vertex): code 0 = labels are the canonical SCC partition."""
    labels = _i32(labels)
    bad = ctypes.c_int64(-1)
    rc = _load().or_check_partition(g.n, _i32(g.out_off).ctypes.data, _i32(g.out_adj).ctypes.data,
                                    _i32(g.in_off).ctypes.data, _i32(g.in_adj).ctypes.data, labels.ctypes.data,
                                    ctypes.byref(bad))
    return int(rc), int(bad.value)


def bfs_depths(n: int, off, adj, labels, sources) -> np.ndarray:
    """Per source: the largest BFS distance of the label-restricted reach
    (arcs (u,w) with labels[u]==labels[w]>=0), 0 if it reaches only itself."""
    off, adj, labels, sources = _i32(off), _i32(adj), _i32(labels), _i32(sources)
    out = np.zeros(max(len(sources), 1), np.int32)
    rc = _load().or_bfs_depths(n, off.ctypes.data, adj.ctypes.data if len(adj) else None, labels.ctypes.data,
                               len(sources), sources.ctypes.data if len(sources) else None, out.ctypes.data)
    if rc != 0:
        raise ValueError("or_bfs_depths rejected its input: %d" % rc)
    return out[:len(sources)]


def hashbag_sim(batches, lam_log2: int = 10, sigma: int = 50, alpha: float = 0.5, kappa: int = 32,
                seed: int = 1):
    """Sequential hash bag model (Section 3.3).  ``batches``: the keys
    inserted in each round, each round ended by ExtractAll.  Returns a dict:
    ``extracted`` (list of int64 arrays, slot order), ``prefix`` (used prefix
    per round), ``advances`` (rows (chunk, load, cause) for every move of the
    current chunk; cause 0 = sigma samples, 1 = probe limit)."""
    arrs = [np.asarray(b, dtype=np.int64).reshape(-1) for b in batches]
    keys = np.ascontiguousarray(np.concatenate(arrs) if arrs else np.zeros(0, np.int64))
    starts = np.zeros(len(arrs) + 1, np.int64)
    starts[1:] = np.cumsum([len(a) for a in arrs])
    n = int(keys.size)
    out = np.zeros(max(n, 1), np.int64)
    prefix = np.zeros(max(len(arrs), 1), np.int64)
    cap = 4096
    while True:
        ch = np.zeros(cap, np.int32)
        ld = np.zeros(cap, np.float64)
        cz = np.zeros(cap, np.int32)
        na = ctypes.c_int64(0)
        rc = _load().or_hashbag_sim(n, keys.ctypes.data if n else None, len(arrs), starts.ctypes.data, lam_log2,
                                    sigma, alpha, kappa, seed, out.ctypes.data if n else None, prefix.ctypes.data,
                                    ch.ctypes.data, ld.ctypes.data, cz.ctypes.data, cap, ctypes.byref(na))
        if rc != 0:
            raise RuntimeError("or_hashbag_sim failed: %d" % rc)
        if na.value <= cap:
            break
        cap = int(na.value)
    k = int(na.value)
    ext = [out[starts[q]:starts[q + 1]].copy() for q in range(len(arrs))]
    return {"extracted": ext, "prefix": prefix[:len(arrs)].copy(),
            "advances": [(int(ch[i]), float(ld[i]), int(cz[i])) for i in range(k)]}


def hashbag_model(inserted_batches, **kw):
    """ExtractAll's output for each round (sorted), as the sequential model of
    Section 3.3 produces it: after any sequence of Inserts, ExtractAll returns
    exactly the inserted multiset (no dedupe)."""
    sim = hashbag_sim(inserted_batches, **kw)
    return [np.sort(e) for e in sim["extracted"]]


def policy_forward(weights: np.ndarray, feats: np.ndarray, n_in: int = 5, hidden: int = 32, n_out: int = 8):
    """Float32 forward of the 3-layer MLP (n_in -> hidden -> hidden -> n_out),
    ReLU between layers.  ``weights`` is the flat blob
    [W1 (hidden x n_in), b1, W2 (hidden x hidden), b2, W3 (n_out x hidden), b3]."""
    w = np.asarray(weights, dtype=np.float32)
    x = np.asarray(feats, dtype=np.float32)
    o = 0

    def take(r, c):
        nonlocal o
        a = w[o:o + r * c].reshape(r, c)
        o += r * c
        return a

    W1 = take(hidden, n_in)
    b1 = take(1, hidden)[0]
    W2 = take(hidden, hidden)
    b2 = take(1, hidden)[0]
    W3 = take(n_out, hidden)
    b3 = take(1, n_out)[0]
    h = np.maximum(x @ W1.T + b1, np.float32(0))
    h = np.maximum(h @ W2.T + b2, np.float32(0))
    return (h @ W3.T + b3).astype(np.float32)
