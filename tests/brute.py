"""Brute-force references used to pin the oracle on tiny inputs.

Reflexive-transitive closure by Warshall's algorithm on a dense boolean
matrix: u and v share an SCC iff u reaches v and v reaches u.  Independent of
the oracle's code (no shared helpers), vectorised with numpy.
"""
import numpy as np


def closure(n, off, adj, keep=None):
    """R[u, v] = True iff u reaches v (reflexive).  keep(u, w) filters arcs."""
    R = np.eye(n, dtype=bool)
    for u in range(n):
        for e in range(off[u], off[u + 1]):
            w = adj[e]
            if keep is None or keep(u, w):
                R[u, w] = True
    for k in range(n):
        R |= np.outer(R[:, k], R[k, :])
    return R


def scc_min_labels(n, off, adj):
    if n == 0:
        return np.zeros(0, np.int32)
    R = closure(n, off, adj)
    M = R & R.T
    return np.argmax(M, axis=1).astype(np.int32)  # first True = min id in the SCC


def reach_pairs(n, off, adj, labels, sources):
    def keep(u, w):
        return labels[u] == labels[w] and labels[u] >= 0
    R = closure(n, off, adj, keep)
    out = []
    for j, s in enumerate(sources):
        for v in np.nonzero(R[s])[0]:
            out.append((int(v), j))
    return np.array(out, dtype=np.int32).reshape(-1, 2)
