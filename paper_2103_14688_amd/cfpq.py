"""Thin Python binding of the C ABI in include/cfpq.h (argument marshalling
only).  Every step of the query runs in libcfpq.so's HIP kernels; if the
library is missing this module raises instead of computing anything itself.

PyTorch is used for plumbing only: device memory comes from its caching
allocator (through the allocator hooks of the ABI) and work is issued on the
current torch stream unless another stream is given.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfpq.so")

OK, ERR_INVALID, ERR_OOM, ERR_DEVICE, ERR_NOT_FOUND, ERR_BUFFER, ERR_LIMIT, ERR_REJECTED = 0, -1, -2, -3, -4, -5, -6, -7
ADD_INVERSES = 1
DEVICE_PTRS = 2
STRATEGY_AUTO, STRATEGY_LEVELS, STRATEGY_FUSED, STRATEGY_CONDENSED, STRATEGY_PEREDGE = 0, 1, 2, 3, 4
NT_AUTO, NT_ROWS, NT_MFMA = 0, 1, 2

_STATUS = {0: "OK", -1: "INVALID", -2: "OOM", -3: "DEVICE", -4: "NOT_FOUND", -5: "BUFFER", -6: "LIMIT",
           -7: "REJECTED"}

EXPORTS = [
    "cfpq_graph_create", "cfpq_graph_info", "cfpq_graph_destroy", "cfpq_rsm_create", "cfpq_rsm_destroy",
    "cfpq_query", "cfpq_query_batch", "cfpq_result_count", "cfpq_result_hash", "cfpq_result_bitmap",
    "cfpq_result_pairs", "cfpq_result_block", "cfpq_result_stats", "cfpq_result_profile", "cfpq_extract_path",
    "cfpq_result_destroy", "cfpq_last_error", "cfpq_version", "cfpq_paths_open", "cfpq_paths_next",
    "cfpq_paths_close", "cfpq_query_noalloc",
]


class CfpqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_CACHED_FN = ctypes.CFUNCTYPE(ctypes.c_size_t, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p), ("cached", _CACHED_FN)]


class QueryOpts(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_uint32), ("max_iters", ctypes.c_uint32), ("keep_rank", ctypes.c_uint32),
                ("keep_blocks", ctypes.c_uint32), ("tile_words", ctypes.c_uint32), ("profile", ctypes.c_uint32),
                ("nt_mode", ctypes.c_uint32), ("recompute", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("alloc", ctypes.POINTER(Allocator)),
                ("src_mask", ctypes.c_void_p), ("dst_mask", ctypes.c_void_p)]


_lib = None


def load():
    """Load libcfpq.so (built by paper_2103_14688_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          f"(python -m paper_2103_14688_amd.build); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "cfpq_graph_create": [u32, u32, vp, vp, vp, u64, u32, P(Allocator), vp, P(vp)],
        "cfpq_graph_info": [vp, P(u32), P(u32), P(u64)],
        "cfpq_rsm_create": [u32, u32, u32, vp, vp, vp, vp, vp, vp, u32, u32, P(vp)],
        "cfpq_query": [vp, vp, P(QueryOpts), P(vp)],
        "cfpq_query_batch": [P(vp), P(vp), u32, P(QueryOpts), P(vp)],
        "cfpq_result_count": [vp, u32, P(u64)],
        "cfpq_result_hash": [vp, u32, P(u64)],
        "cfpq_result_bitmap": [vp, u32, vp, u64, ctypes.c_int],
        "cfpq_result_pairs": [vp, u32, vp, u64, P(u64)],
        "cfpq_result_block": [vp, u32, u32, vp, u64],
        "cfpq_result_stats": [vp, P(u32), vp, u32, P(ctypes.c_double)],
        "cfpq_result_profile": [vp, u32, P(u64), P(ctypes.c_double), P(u64)],
        "cfpq_extract_path": [vp, u32, u32, u32, vp, u64, P(u64)],
        "cfpq_paths_open": [vp, u32, u32, u32, u32, P(vp)],
        "cfpq_paths_next": [vp, vp, u64, P(u64)],
        "cfpq_query_noalloc": [vp, vp, u32, vp, u64, P(u64), P(u32), vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("cfpq_graph_destroy", "cfpq_rsm_destroy", "cfpq_result_destroy", "cfpq_paths_close"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = None
    lib.cfpq_last_error.restype = ctypes.c_char_p
    lib.cfpq_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != OK:
        raise CfpqError(status, load().cfpq_last_error().decode(errors="replace"))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


# ---------------------------------------------------------------------------
# torch plumbing: caching allocator and streams
# ---------------------------------------------------------------------------
_torch_alloc = None


def torch_allocator():
    """Allocator hooks backed by torch.cuda's caching allocator."""
    global _torch_alloc
    if _torch_alloc is None:
        import torch

        def _alloc(size, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), torch.cuda.current_device(),
                                                          stream if stream else 0)
            except Exception:
                return None

        cuda = torch.cuda

        def _free(ptr, size, stream, ctx):
            # at interpreter exit torch may already be torn down; the process
            # releases the memory then anyway
            try:
                cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        def _cached(ctx):
            # reserved but unallocated, less the free pieces of segments that
            # still hold live blocks: what torch hands out again, or releases
            # to the device when an allocation needs it
            try:
                st = torch.cuda.memory_stats(torch.cuda.current_device())
                free_blocks = st.get("reserved_bytes.all.current", 0) - st.get("allocated_bytes.all.current", 0)
                return max(0, free_blocks - st.get("inactive_split_bytes.all.current", 0))
            except Exception:
                return 0

        a = Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None, _CACHED_FN(_cached))
        _torch_alloc = a
    return _torch_alloc


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
# ABI calls (same names as the C functions)
# ---------------------------------------------------------------------------

def cfpq_graph_create(n, n_labels, src, label, dst, flags=0, alloc=None, stream=None):
    """Edge arrays: host arrays (anything numpy converts), or, with
    DEVICE_PTRS in flags, int32/uint32 device tensors (torch) of equal length."""
    lib = load()
    if flags & DEVICE_PTRS:
        import torch
        arrs = [x.contiguous() for x in (src, label, dst)]
        if any(x.dtype not in (torch.int32, torch.uint32) or not x.is_cuda for x in arrs):
            raise ValueError("DEVICE_PTRS needs 32-bit integer device tensors")
        m = arrs[0].numel()
        if any(x.numel() != m for x in arrs):
            raise ValueError("edge arrays differ in length")
        ptrs = [ctypes.c_void_p(x.data_ptr()) for x in arrs]
    else:
        src, label, dst = _u32(src), _u32(label), _u32(dst)
        if not (len(src) == len(label) == len(dst)):
            raise ValueError("edge arrays differ in length")
        m = len(src)
        ptrs = [_ptr(src), _ptr(label), _ptr(dst)]
    out = ctypes.c_void_p()
    _check(lib.cfpq_graph_create(n, n_labels, ptrs[0], ptrs[1], ptrs[2], m, flags,
                                 ctypes.byref(alloc) if alloc is not None else None, stream, ctypes.byref(out)))
    return out.value


def cfpq_graph_info(g):
    n, L, m = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    _check(load().cfpq_graph_info(g, ctypes.byref(n), ctypes.byref(L), ctypes.byref(m)))
    return n.value, L.value, m.value


def cfpq_graph_destroy(g):
    load().cfpq_graph_destroy(g)


def cfpq_rsm_create(n_states, n_terminals, n_boxes, box_start, state_box, is_final, t_src, t_sym, t_dst,
                    start_box=0):
    lib = load()
    box_start, state_box = _u32(box_start), _u32(state_box)
    is_final = np.ascontiguousarray(np.asarray(is_final, dtype=np.uint8))
    t_src, t_sym, t_dst = _u32(t_src), _u32(t_sym), _u32(t_dst)
    out = ctypes.c_void_p()
    _check(lib.cfpq_rsm_create(n_states, n_terminals, n_boxes, _ptr(box_start), _ptr(state_box), _ptr(is_final),
                               _ptr(t_src), _ptr(t_sym), _ptr(t_dst), len(t_src), start_box, ctypes.byref(out)))
    return out.value


def cfpq_rsm_destroy(r):
    load().cfpq_rsm_destroy(r)


def vertex_mask(mask, n):
    """A vertex mask as ceil(n/64) uint64 words: from a bool array of length n
    or from such words; None stays None."""
    if mask is None:
        return None
    m = np.asarray(mask)
    words = (n + 63) // 64
    if m.dtype == np.bool_:
        if m.shape != (n,):
            raise ValueError("a boolean mask needs one entry per vertex")
        bits = np.zeros(words * 64, dtype=np.uint8)
        bits[:n] = m
        return np.ascontiguousarray(np.packbits(bits, bitorder="little").view(np.uint64))
    m = np.ascontiguousarray(m, dtype=np.uint64)
    if m.shape != (words,):
        raise ValueError(f"a word mask needs {words} uint64 words")
    return m


def make_opts(strategy=STRATEGY_AUTO, max_iters=0, keep_rank=False, keep_blocks=False, tile_words=0,
              stream=None, alloc=None, profile=False, nt_mode=NT_AUTO, src_mask=None, dst_mask=None,
              recompute=False):
    """Options struct; masks must be word arrays (vertex_mask) that the caller
    keeps alive until the call returns."""
    o = QueryOpts(strategy, max_iters, int(keep_rank), int(keep_blocks), tile_words, int(profile), int(nt_mode),
                  int(recompute), stream, None, None, None)
    if alloc is not None:
        o.alloc = ctypes.pointer(alloc)
    if src_mask is not None:
        o.src_mask = src_mask.ctypes.data
    if dst_mask is not None:
        o.dst_mask = dst_mask.ctypes.data
    return o


def cfpq_query(g, r, opts=None):
    out = ctypes.c_void_p()
    _check(load().cfpq_query(g, r, ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return out.value


def cfpq_query_noalloc(g, r, box, dst, stream=None):
    """The fused fixpoint without device allocation: box's relation into dst,
    a torch CUDA tensor of n * ceil(n/64) int64/uint64 words (row-major
    bitmap).  Returns (pairs, iterations)."""
    pairs, it = ctypes.c_uint64(), ctypes.c_uint32()
    _check(load().cfpq_query_noalloc(g, r, box, ctypes.c_void_p(dst.data_ptr()), dst.numel(), ctypes.byref(pairs),
                                     ctypes.byref(it), stream))
    return pairs.value, it.value


def cfpq_query_batch(graphs, rsms, opts=None):
    k = len(graphs)
    G = (ctypes.c_void_p * k)(*graphs)
    R = (ctypes.c_void_p * k)(*rsms)
    out = (ctypes.c_void_p * k)()
    _check(load().cfpq_query_batch(G, R, k, ctypes.byref(opts) if opts is not None else None, out))
    return [out[i] for i in range(k)]


def cfpq_result_count(res, box):
    c = ctypes.c_uint64()
    _check(load().cfpq_result_count(res, box, ctypes.byref(c)))
    return c.value


def cfpq_result_hash(res, box):
    h = ctypes.c_uint64()
    _check(load().cfpq_result_hash(res, box, ctypes.byref(h)))
    return h.value


def cfpq_result_bitmap(res, box, n, dst=None):
    """Row-major bitmap as numpy uint64 [n, ceil(n/64)]; or, if dst is a
    torch CUDA tensor of that many int64/uint64 words, filled on the device."""
    words = (n + 63) // 64
    if dst is not None:
        _check(load().cfpq_result_bitmap(res, box, ctypes.c_void_p(dst.data_ptr()), dst.numel(), 1))
        return dst
    out = np.zeros((n, words), dtype=np.uint64)
    _check(load().cfpq_result_bitmap(res, box, _ptr(out), out.size, 0))
    return out


def cfpq_result_pairs(res, box):
    lib = load()
    cnt = ctypes.c_uint64()
    st = lib.cfpq_result_pairs(res, box, None, 0, ctypes.byref(cnt))
    if st not in (OK, ERR_BUFFER):
        _check(st)
    out = np.zeros((max(1, cnt.value), 2), dtype=np.uint32)
    _check(lib.cfpq_result_pairs(res, box, _ptr(out), cnt.value, ctypes.byref(cnt)))
    return out[: cnt.value]


def cfpq_result_block(res, q_start, q_final, n):
    out = np.zeros((n, (n + 63) // 64), dtype=np.uint64)
    _check(load().cfpq_result_block(res, q_start, q_final, _ptr(out), out.size))
    return out


def cfpq_result_stats(res, cap=4096):
    it = ctypes.c_uint32()
    ms = ctypes.c_double()
    d = np.zeros(cap, dtype=np.uint64)
    _check(load().cfpq_result_stats(res, ctypes.byref(it), _ptr(d), cap, ctypes.byref(ms)))
    return it.value, d[: min(it.value, cap)].tolist(), ms.value


KERNEL_SEED, KERNEL_LEVEL, KERNEL_WRITEBACK, KERNEL_COND_LEVEL, KERNEL_COND_SCC, KERNEL_NT_MFMA, KERNEL_NT_SPARSE, \
    KERNEL_ELL, KERNEL_NT_DENSE = 0, 1, 2, 3, 4, 5, 6, 7, 8


def cfpq_result_profile(res, kind):
    """(launches, summed ms, algorithmic bytes) of one kernel kind."""
    n, ms, by = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint64()
    _check(load().cfpq_result_profile(res, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def cfpq_extract_path(res, box, u, v):
    lib = load()
    n = ctypes.c_uint64()
    st = lib.cfpq_extract_path(res, box, u, v, None, 0, ctypes.byref(n))
    if st == OK:
        return np.zeros((0, 3), dtype=np.uint32)
    if st != ERR_BUFFER:
        _check(st)
    out = np.zeros((n.value, 3), dtype=np.uint32)
    _check(lib.cfpq_extract_path(res, box, u, v, _ptr(out), n.value, ctypes.byref(n)))
    return out


def cfpq_paths_open(res, box, u, v, max_edges):
    out = ctypes.c_void_p()
    _check(load().cfpq_paths_open(res, box, u, v, max_edges, ctypes.byref(out)))
    return out.value


def cfpq_paths_next(it, cap=64):
    """The next path as an (edges, 3) array, or None when none is left."""
    lib = load()
    n = ctypes.c_uint64()
    while True:
        buf = np.zeros((cap, 3), dtype=np.uint32)
        st = lib.cfpq_paths_next(it, _ptr(buf), cap, ctypes.byref(n))
        if st == OK:
            return buf[:n.value].copy()
        if st == ERR_NOT_FOUND:
            return None
        if st != ERR_BUFFER:
            _check(st)
        cap = int(n.value)


def cfpq_paths_close(it):
    load().cfpq_paths_close(it)


def cfpq_result_destroy(res):
    load().cfpq_result_destroy(res)


def cfpq_version():
    return load().cfpq_version().decode()


# ---------------------------------------------------------------------------
# small owning wrappers
# ---------------------------------------------------------------------------

class Graph:
    """Resident graph handle.  labels: names, label id = index."""

    def __init__(self, n, src, lbl, dst, labels, flags=0, use_torch=True, stream=None):
        self.n = int(n)
        self.labels = list(labels)
        self._alloc = torch_allocator() if use_torch else None
        if stream is None and use_torch:
            stream = current_stream()
        self.h = cfpq_graph_create(self.n, len(self.labels), src, lbl, dst, flags, self._alloc, stream)

    @classmethod
    def from_synth(cls, g, **kw):
        return cls(g.n, g.src, g.lbl, g.dst, g.labels, **kw)

    def info(self):
        return cfpq_graph_info(self.h)

    def close(self):
        if self.h:
            cfpq_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Query:
    """RSM handle built from an rsm.RSM."""

    def __init__(self, rsm):
        self.rsm = rsm
        self.h = cfpq_rsm_create(rsm.n_states, rsm.n_terminals, rsm.n_boxes, rsm.box_start, rsm.state_box,
                                 rsm.is_final, rsm.t_src, rsm.t_sym, rsm.t_dst, rsm.start_box)

    def close(self):
        if self.h:
            cfpq_rsm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Result:
    def __init__(self, h, graph, query):
        self.h, self.n, self.query = h, graph.n, query
        self._graph = graph     # keeps the allocator alive

    def box(self, name):
        return self.query.rsm.box(name) if isinstance(name, str) else int(name)

    def count(self, box=0):
        return cfpq_result_count(self.h, self.box(box))

    def hash(self, box=0):
        return cfpq_result_hash(self.h, self.box(box))

    def bitmap(self, box=0, dst=None):
        return cfpq_result_bitmap(self.h, self.box(box), self.n, dst)

    def pairs(self, box=0):
        return cfpq_result_pairs(self.h, self.box(box))

    def block(self, q_start, q_final):
        return cfpq_result_block(self.h, q_start, q_final, self.n)

    def stats(self):
        return cfpq_result_stats(self.h)

    def profile(self, kind):
        return cfpq_result_profile(self.h, kind)

    def extract_path(self, u, v, box=0):
        return cfpq_extract_path(self.h, self.box(box), u, v)

    def paths(self, u, v, max_edges, box=0):
        """All paths u -> v with at most max_edges edges whose words the box
        derives, each once, shortest first (a generator over (k, 3) arrays)."""
        it = cfpq_paths_open(self.h, self.box(box), u, v, max_edges)
        try:
            while True:
                p = cfpq_paths_next(it)
                if p is None:
                    return
                yield p
        finally:
            cfpq_paths_close(it)

    def close(self):
        if self.h:
            cfpq_result_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query(graph, q, strategy=STRATEGY_AUTO, max_iters=0, keep_rank=False, keep_blocks=False, tile_words=0,
          stream=None, profile=False, nt_mode=NT_AUTO, src_mask=None, dst_mask=None, recompute=False):
    """src_mask / dst_mask: bool arrays of length n or ceil(n/64) uint64
    words restricting the start box's sources / targets (None = all)."""
    if stream is None:
        stream = current_stream()
    sm, dm = vertex_mask(src_mask, graph.n), vertex_mask(dst_mask, graph.n)
    o = make_opts(strategy, max_iters, keep_rank, keep_blocks, tile_words, stream, graph._alloc, profile, nt_mode,
                  sm, dm, recompute)
    return Result(cfpq_query(graph.h, q.h, o), graph, q)


def query_noalloc(graph, q, box=0, dst=None, stream=None):
    """cfpq_query_noalloc on the current torch stream; dst defaults to a new
    tensor (allocated here by torch, not by the library).  Returns
    (bitmap tensor [n, ceil(n/64)], pairs, iterations)."""
    import torch
    if stream is None:
        stream = current_stream()
    if dst is None:
        dst = torch.empty((graph.n, (graph.n + 63) // 64), dtype=torch.int64, device="cuda")
    b = q.rsm.box(box) if isinstance(box, str) else int(box)
    pairs, it = cfpq_query_noalloc(graph.h, q.h, b, dst, stream)
    return dst, pairs, it


def query_batch(graphs, queries, strategy=STRATEGY_AUTO, max_iters=0, keep_rank=False, keep_blocks=False,
                tile_words=0, stream=None):
    if stream is None:
        stream = current_stream()
    o = make_opts(strategy, max_iters, keep_rank, keep_blocks, tile_words, stream,
                  graphs[0]._alloc if graphs else None)
    hs = cfpq_query_batch([g.h for g in graphs], [q.h for q in queries], o)
    return [Result(h, g, q) for h, g, q in zip(hs, graphs, queries)]
