"""hipscc: SCC and reachability on one MI355X (gfx950) via a C-ABI HIP library.

Thin Python binding: it only marshals torch device tensors (memory and
streams) into the C ABI of ``include/hipscc.h``; every step of the method runs
in the library's HIP kernels.  Importing works without a GPU; calls need one
and raise if the library is not built.

    import paper_2303_04934_amd as scc
    dg = scc.to_device(graph)          # graph: n, m, out_off, out_adj, in_off, in_adj
    labels = scc.scc_labels(dg)        # int32 [n], min vertex id of each SCC
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _native
from ._native import POLICY_FLOATS, STATUS_NAMES, Options, Stats

__all__ = ["SccError", "DeviceGraph", "to_device", "default_options", "scc_labels", "scc_labels_static", "scc_cc", "scc_le_lists", "scc_reach",
           "scc_labels_batched", "bag_selftest", "bag_stats", "policy_load", "policy_eval", "trace_read", "version",
           "POLICY_FLOATS", "TRACE_FIELDS"]

TRACE_FIELDS = _native.TRACE_FIELDS


class SccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


def _torch():
    import torch
    return torch


@dataclass
class DeviceGraph:
    n: int
    m: int
    out_off: object
    out_adj: object
    in_off: object
    in_adj: object

    def c_struct(self):
        return _native.Graph(self.n, self.m, self.out_off.data_ptr(), self.out_adj.data_ptr() if self.m else 0,
                             self.in_off.data_ptr(), self.in_adj.data_ptr() if self.m else 0)


def to_device(g, device="cuda") -> DeviceGraph:
    """Copy a host graph (numpy int32 CSR + transposed CSR) to device tensors."""
    torch = _torch()

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
    return DeviceGraph(int(g.n), int(g.m), up(g.out_off), up(g.out_adj), up(g.in_off), up(g.in_adj))


_contexts = {}


def _ctx(device_index: int, stream_handle: int):
    key = (device_index, stream_handle)
    c = _contexts.get(key)
    if c is None:
        lib = _native.load()
        p = ctypes.c_void_p()
        rc = lib.scc_create(ctypes.byref(p), device_index, ctypes.c_void_p(stream_handle))
        if rc != 0:
            raise SccError(rc, "scc_create failed on device %d" % device_index)
        c = _contexts[key] = p
    return c


def _current(t):
    torch = _torch()
    dev = t.device.index if t.device.index is not None else torch.cuda.current_device()
    s = torch.cuda.current_stream(dev).cuda_stream
    return _ctx(dev, s)


def _check(lib, ctx, rc):
    if rc != 0:
        raise SccError(rc, lib.scc_last_error(ctx).decode(errors="replace"))


def default_options(**kw) -> Options:
    o = Options()
    _native.load().scc_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def version() -> str:
    return _native.load().scc_version().decode()


def scc_labels(dg: DeviceGraph, options: Options | None = None, return_stats: bool = False, out=None):
    """SCC labels (min vertex id per SCC) of a device graph, int32 tensor [n]."""
    torch = _torch()
    lib = _native.load()
    ctx = _current(dg.out_off)
    if out is None:
        out = torch.empty(max(dg.n, 1), dtype=torch.int32, device=dg.out_off.device)
    st = Stats()
    g = dg.c_struct()
    rc = lib.scc_labels(ctx, ctypes.byref(g), out.data_ptr(), ctypes.byref(options) if options else None,
                        ctypes.byref(st))
    _check(lib, ctx, rc)
    out = out[:dg.n]
    return (out, st.as_dict()) if return_stats else out


def scc_labels_static(dg: DeviceGraph, out, options: Options | None = None, return_stats: bool = False):
    """scc_labels without device allocation: scratch comes from the library's
    fixed per-device array (see scc_labels_static in hipscc.h).  ``out`` is a
    caller-allocated int32 device tensor of at least n elements."""
    lib = _native.load()
    ctx = _current(dg.out_off)
    st = Stats()
    g = dg.c_struct()
    rc = lib.scc_labels_static(ctx, ctypes.byref(g), out.data_ptr(), ctypes.byref(options) if options else None,
                               ctypes.byref(st))
    _check(lib, ctx, rc)
    res = out[:dg.n]
    return (res, st.as_dict()) if return_stats else res


def scc_cc(dg: DeviceGraph, options: Options | None = None, return_stats: bool = False, out=None):
    """Connected components (LDD-UF-JTB): smallest vertex id of each vertex's
    weakly connected component, int32 tensor [n].  Reads the out-CSR only."""
    torch = _torch()
    lib = _native.load()
    ctx = _current(dg.out_off)
    if out is None:
        out = torch.empty(max(dg.n, 1), dtype=torch.int32, device=dg.out_off.device)
    st = Stats()
    g = dg.c_struct()
    rc = lib.scc_cc(ctx, ctypes.byref(g), out.data_ptr(), ctypes.byref(options) if options else None,
                    ctypes.byref(st))
    _check(lib, ctx, rc)
    out = out[:dg.n]
    return (out, st.as_dict()) if return_stats else out


def scc_le_lists(dg: DeviceGraph, options: Options | None = None, capacity: int | None = None,
                 return_stats: bool = False):
    """Least-element lists: (order int32[n], loff int64[n+1], src int32[k],
    dist int32[k]) device tensors; see scc_le_lists in hipscc.h."""
    torch = _torch()
    lib = _native.load()
    dev = dg.out_off.device
    ctx = _current(dg.out_off)
    n = dg.n
    if capacity is None:
        capacity = max(64, 8 * n)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    loff = torch.empty(n + 1, dtype=torch.int64, device=dev)
    src = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    dist = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    cnt = ctypes.c_int64(0)
    st = Stats()
    g = dg.c_struct()
    rc = lib.scc_le_lists(ctx, ctypes.byref(g), order.data_ptr(), loff.data_ptr(), src.data_ptr(), dist.data_ptr(),
                          capacity, ctypes.byref(cnt), ctypes.byref(options) if options else None, ctypes.byref(st))
    if rc == _native.SCC_ECAPACITY:
        return scc_le_lists(dg, options, int(cnt.value), return_stats)
    _check(lib, ctx, rc)
    k = int(cnt.value)
    out = (order[:n], loff, src[:k], dist[:k])
    return (out, st.as_dict()) if return_stats else out


def scc_reach(dg: DeviceGraph, sources, labels, direction: int = 0, capacity: int | None = None,
              options: Options | None = None, return_stats: bool = False):
    """Reachability pairs (vertex, source index) as an int32 tensor [count, 2],
    sorted ascending by (source index, vertex) on the device.  Arcs are used
    only between equal, non-negative labels."""
    torch = _torch()
    lib = _native.load()
    dev = dg.out_off.device
    sources = torch.as_tensor(sources, dtype=torch.int32, device=dev).contiguous()
    labels = torch.as_tensor(labels, dtype=torch.int32, device=dev).contiguous()
    ctx = _current(dg.out_off)
    k = int(sources.numel())
    if capacity is None:
        capacity = max(16, k * max(dg.n, 1)) if k * max(dg.n, 1) < (1 << 26) else (1 << 26)
    pairs = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=dev)
    cnt = ctypes.c_int64(0)
    st = Stats()
    g = dg.c_struct()
    rc = lib.scc_reach(ctx, ctypes.byref(g), direction, sources.data_ptr() if k else None, k,
                       labels.data_ptr() if k else None, pairs.data_ptr(), capacity, ctypes.byref(cnt),
                       ctypes.byref(options) if options else None, ctypes.byref(st))
    if rc == _native.SCC_ECAPACITY:
        need = int(cnt.value)
        return scc_reach(dg, sources, labels, direction, need, options, return_stats)
    _check(lib, ctx, rc)
    out = pairs[:cnt.value]
    return (out, st.as_dict()) if return_stats else out


def scc_labels_batched(vtx_base, arc_base, out_off, out_adj, in_off, in_adj, options: Options | None = None,
                       return_stats: bool = False):
    """SCC labels of many graphs at once (local ids); see scc_labels_batched in hipscc.h."""
    torch = _torch()
    lib = _native.load()
    vb = np.ascontiguousarray(vtx_base, dtype=np.int64)
    ab = np.ascontiguousarray(arc_base, dtype=np.int64)
    G = len(vb) - 1
    ctx = _current(out_off)
    out = torch.empty(max(int(vb[-1]), 1), dtype=torch.int32, device=out_off.device)
    st = Stats()
    rc = lib.scc_labels_batched(ctx, G, vb.ctypes.data, ab.ctypes.data, out_off.data_ptr(),
                                out_adj.data_ptr() if out_adj.numel() else None, in_off.data_ptr(),
                                in_adj.data_ptr() if in_adj.numel() else None, out.data_ptr(),
                                ctypes.byref(options) if options else None, ctypes.byref(st))
    _check(lib, ctx, rc)
    out = out[:int(vb[-1])]
    return (out, st.as_dict()) if return_stats else out


def bag_selftest(keys, rounds: int = 1, options: Options | None = None, return_stats: bool = False):
    """Insert every key into the hash bag (round robin over `rounds` rounds) and
    return what the ExtractAll calls returned (uint64 keys as int64)."""
    torch = _torch()
    lib = _native.load()
    keys = keys.contiguous()
    ctx = _current(keys)
    n = int(keys.numel())
    out = torch.empty(max(n, 1), dtype=torch.int64, device=keys.device)
    cnt = ctypes.c_int64(0)
    st = Stats()
    rc = lib.scc_bag_selftest(ctx, keys.data_ptr() if n else None, n, rounds, out.data_ptr(), ctypes.byref(cnt),
                              ctypes.byref(options) if options else None, ctypes.byref(st))
    _check(lib, ctx, rc)
    out = out[:cnt.value]
    return (out, st.as_dict()) if return_stats else out


def bag_stats(device_index: int = 0):
    """Statistics of the last bag_selftest on the current stream's context:
    (rows [r, 4] of (round, chunk, load, cause) for every chunk left during a
    round, cause 0 = samples reached sigma, 1 = probe limit; used prefix per
    round)."""
    torch = _torch()
    lib = _native.load()
    ctx = _ctx(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    nr, nq = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib, ctx, lib.scc_bag_stats(ctx, None, 0, ctypes.byref(nr), None, 0, ctypes.byref(nq)))
    rows = np.zeros((max(int(nr.value), 1), 4), np.float64)
    prefix = np.zeros(max(int(nq.value), 1), np.int64)
    _check(lib, ctx, lib.scc_bag_stats(ctx, rows.ctypes.data, int(nr.value), ctypes.byref(nr), prefix.ctypes.data,
                                       int(nq.value), ctypes.byref(nq)))
    return rows[:int(nr.value)], prefix[:int(nq.value)]


def trace_read(device_index: int = 0):
    """Per-round trace rows of the last call made with options.trace=1 on the
    current stream's context, as a float32 array [rows, TRACE_FIELDS]."""
    torch = _torch()
    lib = _native.load()
    ctx = _ctx(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    n = ctypes.c_int64(0)
    _check(lib, ctx, lib.scc_trace_read(ctx, None, 0, ctypes.byref(n)))
    out = np.empty((max(int(n.value), 1), TRACE_FIELDS), np.float32)
    _check(lib, ctx, lib.scc_trace_read(ctx, out.ctypes.data, int(n.value), ctypes.byref(n)))
    return out[:int(n.value)]


def policy_load(weights, device_index: int = 0):
    torch = _torch()
    lib = _native.load()
    w = np.ascontiguousarray(weights, dtype=np.float32)
    ctx = _ctx(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    _check(lib, ctx, lib.scc_policy_load(ctx, w.ctypes.data, w.size))


def policy_eval(feats, device_index: int = 0):
    torch = _torch()
    lib = _native.load()
    x = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 5)
    out = np.empty((x.shape[0], 8), np.float32)
    ctx = _ctx(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    _check(lib, ctx, lib.scc_policy_eval(ctx, x.ctypes.data, x.shape[0], out.ctypes.data))
    return out
