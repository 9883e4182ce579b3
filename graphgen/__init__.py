"""Seeded synthetic digraphs for the SCC library and its oracle.

Input side only: this package builds int32 CSR + transposed CSR arrays (host
numpy) and holds none of the SCC method's arithmetic.  Both the GPU path and
the sequential oracle consume what it returns.

The workload shapes stand in for the paper's evaluation graphs (Section 6:
lattices, social/web graphs, k-NN graphs), which are not available here:

* ``torus``/``grid``  -- 2-D lattice, every neighbour arc kept with p;
* ``lattice_oriented`` -- the paper's SQR/REC (mode 0) and SQR'/REC' (mode 1)
  tori with randomly oriented edges (Section 6);
* ``rmat``            -- R-MAT (a, b, c, d) digraph, dedup, random ids;
* ``knn``             -- directed k-NN graph of a 3-D Gaussian mixture;
* ``batched``         -- many graphs with log-uniform sizes, family mixed.

The C source (``graphgen.c``) is compiled with gcc by :func:`build`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("off", ctypes.POINTER(ctypes.c_int32)), ("adj", ctypes.POINTER(ctypes.c_int32))]


def build(force: bool = True) -> str:
    """Compile the generator library in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.gg_lattice.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_uint64, P(_Csr)]
        lib.gg_lattice_oriented.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, P(_Csr)]
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, P(_Csr)]
        lib.gg_knn.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                               ctypes.c_uint64, P(_Csr), ctypes.c_void_p]
        lib.gg_transpose.argtypes = [P(_Csr), P(_Csr)]
        lib.gg_from_arcs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int, P(_Csr)]
        lib.gg_free.argtypes = [P(_Csr)]
        lib.gg_rnd.argtypes = [ctypes.c_uint64] * 3
        lib.gg_rnd.restype = ctypes.c_uint64
        lib.gg_unif.argtypes = [ctypes.c_uint64] * 3
        lib.gg_unif.restype = ctypes.c_double
        lib.gg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """A digraph as int32 CSR of out-arcs plus the transposed CSR."""
    n: int
    m: int
    out_off: np.ndarray
    out_adj: np.ndarray
    in_off: np.ndarray
    in_adj: np.ndarray
    name: str = ""

    def nbytes(self) -> int:
        return int(self.out_off.nbytes + self.out_adj.nbytes + self.in_off.nbytes + self.in_adj.nbytes)


def _take(c: _Csr):
    lib = _load()
    n, m = int(c.n), int(c.m)
    off = np.ctypeslib.as_array(c.off, shape=(n + 1,)).copy()
    adj = np.ctypeslib.as_array(c.adj, shape=(max(m, 1),))[:m].copy()
    lib.gg_free(ctypes.byref(c))
    return n, m, off, adj


def _finish(c: _Csr, name: str) -> Graph:
    lib = _load()
    t = _Csr()
    rc = lib.gg_transpose(ctypes.byref(c), ctypes.byref(t))
    if rc != 0:
        lib.gg_free(ctypes.byref(c))
        raise MemoryError("gg_transpose failed (%d)" % rc)
    n, m, off, adj = _take(c)
    _, _, ioff, iadj = _take(t)
    return Graph(n, m, off, adj, ioff, iadj, name)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def lattice(rows: int, cols: int, p: float, seed: int, wrap: bool) -> Graph:
    c = _Csr()
    _check(_load().gg_lattice(rows, cols, 1 if wrap else 0, p, seed, ctypes.byref(c)), "gg_lattice")
    return _finish(c, "%s%dx%d_p%g" % ("torus" if wrap else "grid", rows, cols, p))


def torus(rows: int, cols: int, p: float = 0.5, seed: int = 1000) -> Graph:
    return lattice(rows, cols, p, seed, True)


def grid(rows: int, cols: int, p: float = 0.5, seed: int = 1003) -> Graph:
    return lattice(rows, cols, p, seed, False)


def lattice_oriented(rows: int, cols: int, mode: int, seed: int) -> Graph:
    """The paper's lattices (Section 6), a rows x cols torus: mode 0 = SQR/REC
    (each endpoint draws an orientation for each of its edges, duplicates
    removed), mode 1 = SQR'/REC' (each arc of each edge kept independently
    with probability 0.3)."""
    c = _Csr()
    _check(_load().gg_lattice_oriented(rows, cols, mode, seed, ctypes.byref(c)), "gg_lattice_oriented")
    return _finish(c, "%s%dx%d" % ("olat" if mode == 0 else "olat2_", rows, cols))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1001, permute: bool = True) -> Graph:
    cs = _Csr()
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, seed, 1 if permute else 0, ctypes.byref(cs)), "gg_rmat")
    return _finish(cs, "rmat_s%d_ef%d" % (scale, edge_factor))


def knn(npts: int, ncent: int = 1000, k: int = 5, sigma: float = 0.01, seed: int = 1002,
        return_points: bool = False):
    cs = _Csr()
    pts = np.empty((npts, 3), dtype=np.float64) if return_points else None
    ptr = pts.ctypes.data if pts is not None else None
    _check(_load().gg_knn(npts, ncent, k, sigma, seed, ctypes.byref(cs), ptr), "gg_knn")
    g = _finish(cs, "knn_n%d_c%d_k%d" % (npts, ncent, k))
    return (g, pts) if return_points else g


def from_arcs(n: int, src, dst, dedup: bool = False, name: str = "arcs") -> Graph:
    """CSR + transpose of an explicit arc list (duplicates kept unless dedup)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if len(src) and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("arc endpoint out of range")
    cs = _Csr()
    _check(_load().gg_from_arcs(n, len(src), src.ctypes.data, dst.ctypes.data, 1 if dedup else 0,
                                ctypes.byref(cs)), "gg_from_arcs")
    return _finish(cs, name)


def symmetrize(g: Graph) -> Graph:
    """The symmetric digraph with both arcs of every arc of g (duplicates
    removed): the undirected graphs Section 5 runs connectivity on."""
    src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.out_off))
    return from_arcs(g.n, np.concatenate([src, g.out_adj]), np.concatenate([g.out_adj, src]), dedup=True,
                     name=g.name + "_sym")


def random_digraph(n: int, avg_deg: float, seed: int, self_loops: bool = False) -> Graph:
    """Erdos-Renyi style digraph with about n*avg_deg arcs (duplicates removed)."""
    m0 = int(round(n * avg_deg))
    lib = _load()
    src = np.array([lib.gg_rnd(seed, 30, 2 * i) % max(n, 1) for i in range(m0)], dtype=np.int64) if n else \
        np.zeros(0, np.int64)
    dst = np.array([lib.gg_rnd(seed, 30, 2 * i + 1) % max(n, 1) for i in range(m0)], dtype=np.int64) if n else \
        np.zeros(0, np.int64)
    if not self_loops and m0:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if m0:
        key = np.unique(src * n + dst)
        src, dst = key // n, key % n
    return from_arcs(n, src, dst, name="er_n%d_d%g_s%d" % (n, avg_deg, seed))


def rnd(seed: int, stream: int, idx: int) -> int:
    return int(_load().gg_rnd(seed, stream, idx))


def unif(seed: int, stream: int, idx: int) -> float:
    return float(_load().gg_unif(seed, stream, idx))


# ----------------------------------------------------------------- configs --
CONFIG_NAMES = [
    "torus1000_p0.5",      # 0: 2-D torus 1000x1000, arcs kept with p=0.5
    "rmat_s24_ef16",       # 1: R-MAT scale 24, edge factor 16, (.57,.19,.19,.05)
    "knn_10M_k5",          # 2: 3-D Gaussian-mixture k-NN, 1e7 points, 1000 centres
    "grid10000_p0.5",      # 3: 2-D grid 10000x10000 (no wrap), p=0.5
    "batched4096",         # 4: 4096 mixed graphs, log-uniform sizes in [1e3, 1e6]
    "sqr_10000",           # 5: the paper's SQR, 10^4 x 10^4 torus, random orientations
    "rec_1000x10000",      # 6: the paper's REC, 10^3 x 10^4 torus
    "sqr2_10000",          # 7: the paper's SQR', each arc of an edge kept with p=0.3
    "rec2_1000x10000",     # 8: the paper's REC'
]


def config(i: int, shrink: int = 0) -> Graph:
    """Workload i at full size (shrink=0) or reduced by 2**shrink in n."""
    seed = 1000 + i
    if i == 0:
        side = max(3, int(round(1000 / math.sqrt(2 ** shrink))))
        return torus(side, side, 0.5, seed)
    if i == 1:
        return rmat(24 - shrink, 16, 0.57, 0.19, 0.19, seed, True)
    if i == 2:
        n = max(64, 10_000_000 >> shrink)
        return knn(n, max(1, 1000 >> shrink), 5, 0.01, seed)
    if i == 3:
        side = max(3, int(round(10000 / math.sqrt(2 ** shrink))))
        return grid(side, side, 0.5, seed)
    if i in (5, 7):  # SQR, SQR': 10^4 x 10^4
        side = max(3, int(round(10000 / math.sqrt(2 ** shrink))))
        return lattice_oriented(side, side, 0 if i == 5 else 1, seed)
    if i in (6, 8):  # REC, REC': 10^3 x 10^4
        f = math.sqrt(2 ** shrink)
        return lattice_oriented(max(3, int(round(1000 / f))), max(3, int(round(10000 / f))), 0 if i == 6 else 1, seed)
    raise ValueError("config %d is a batch; use batched()" % i)


def batched_spec(G: int = 4096, seed: int = 1004, lo_exp: float = 3.0, hi_exp: float = 6.0):
    """Per-graph (family, n) for the batched workload; family 0 torus, 1 R-MAT, 2 kNN."""
    spec = []
    for g in range(G):
        u = unif(seed, 20, g)
        n = int(round(10 ** (lo_exp + (hi_exp - lo_exp) * u)))
        fam = min(2, int(unif(seed, 21, g) * 3))
        spec.append((fam, n, rnd(seed, 22, g)))
    return spec


def batched(G: int = 4096, seed: int = 1004, lo_exp: float = 3.0, hi_exp: float = 6.0):
    """List of Graphs for the batched workload (sizes log-uniform in 10**[lo,hi])."""
    return batched_slice(G, seed, lo_exp, hi_exp, 0, G)


def batched_slice(G: int, seed: int, lo_exp: float, hi_exp: float, g0: int, g1: int):
    """Graphs g0..g1-1 of the batched workload (the same graphs batched() returns)."""
    out = []
    for fam, n, gseed in batched_spec(G, seed, lo_exp, hi_exp)[g0:g1]:
        if fam == 0:
            rows = max(3, int(round(math.sqrt(n))))
            cols = max(3, int(round(n / rows)))
            out.append(torus(rows, cols, 0.5, gseed))
        elif fam == 1:
            sc = max(2, int(round(math.log2(n))))
            out.append(rmat(sc, 8, 0.57, 0.19, 0.19, gseed, True))
        else:
            out.append(knn(n, max(1, math.ceil(n / 1e4)), 5, 0.01, gseed))
    return out


def concat(graphs):
    """Concatenate graphs into batched arrays with int64 vertex/arc bases (local ids kept)."""
    G = len(graphs)
    vb = np.zeros(G + 1, np.int64)
    ab = np.zeros(G + 1, np.int64)
    for i, g in enumerate(graphs):
        vb[i + 1] = vb[i] + g.n
        ab[i + 1] = ab[i] + g.m
    # graph g keeps its n_g + 1 local offsets at [vb[g] + g, vb[g+1] + g + 1)
    out_off = np.concatenate([g.out_off for g in graphs]) if G else np.zeros(0, np.int32)
    in_off = np.concatenate([g.in_off for g in graphs]) if G else np.zeros(0, np.int32)
    out_adj = np.concatenate([g.out_adj for g in graphs]) if G else np.zeros(0, np.int32)
    in_adj = np.concatenate([g.in_adj for g in graphs]) if G else np.zeros(0, np.int32)
    return vb, ab, out_off, out_adj, in_off, in_adj
