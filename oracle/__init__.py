"""Plain CPU oracle for CFPQ and RPQ reachability.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package.  The product path never
does, and this package imports nothing from the product package.

What it computes is the plain definition the Kronecker-product algorithm is
proved to reach (Theorem 1; reachability semantics in Sec. 2.1):

    R_N = {(u, v) : some path u..v spells a word derivable from N}

``cfl_reach`` evaluates it with a worklist over the grammar's normal form
(``cfl_oracle.c``); ``cfl_reach_rounds`` evaluates the same normal form as a
least fixpoint of relation equations in semi-naive rounds (larger graphs);
``rpq_rows`` evaluates a regular path query by one breadth-first search per
source over the graph x epsilon-NFA product (Sec. 2.2 and 2.4: RPQ as
automata intersection).  ``pairs_hash`` and ``groups_hash`` give the count
and order-independent hash of pair sets too large to store.

All arithmetic is Boolean or integer; results are exact.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import lang

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

EPS_LABEL = 0xFFFFFFFF


def build(force=True):
    """Compile the C oracle with gcc (plain C, OpenMP over independent sources)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_cfl.restype = ctypes.c_int
        lib.oracle_cfl.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u32p,
                                   ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p, u32p,
                                   ctypes.c_uint32, u32p, u64p, u64p, u64p]
        lib.oracle_cfl_rounds.restype = ctypes.c_int
        lib.oracle_cfl_rounds.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u32p,
                                          ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p, u32p,
                                          ctypes.c_uint32, u32p, u64p, u64p, ctypes.c_int, u32p]
        lib.oracle_pairs_hash.restype = None
        lib.oracle_pairs_hash.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u64p, ctypes.c_int, u64p, u64p]
        lib.oracle_groups_hash.restype = None
        lib.oracle_groups_hash.argtypes = [ctypes.c_uint32, u64p, u32p, ctypes.c_int, u64p, u64p]
        lib.oracle_rpq_rows.restype = ctypes.c_int
        lib.oracle_rpq_rows.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u32p,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p,
                                        ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint32, u32p,
                                        u64p, ctypes.c_int, u64p]
        _lib = lib
    return _lib


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def words(n):
    return (n + 63) // 64


def cfl_reach(n, src, lbl, dst, label_names, grammar, nonterminals=None, bitmaps=True):
    """All-pairs CFL-reachability for every requested nonterminal.

    src/lbl/dst: edge arrays (label ids index label_names).
    grammar: text, see ``lang``.  nonterminals: names to report (default:
    all of the grammar's own nonterminals).
    Returns {name: (count, bitmap or None)}; bitmap is uint64 [n, ceil(n/64)],
    row u, bit v (LSB first) set iff (u, v) is in R_name.
    """
    lib = _load()
    label_ids = {name: i for i, name in enumerate(label_names)}
    n_nt, rules, names = lang.grammar_normal_form(grammar, label_ids)
    want = list(names) if nonterminals is None else list(nonterminals)
    out_nt = _u32([names.index(a) for a in want])
    src, lbl, dst = _u32(src), _u32(lbl), _u32(dst)
    kind = _u32([r[0] for r in rules])
    lhs = _u32([r[1] for r in rules])
    x = _u32([r[2] for r in rules])
    y = _u32([r[3] for r in rules])
    w = words(n)
    bits = np.zeros((len(want), n, w), dtype=np.uint64) if bitmaps else None
    counts = np.zeros(len(want), dtype=np.uint64)
    facts = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_cfl(n, len(src), _p32(src), _p32(lbl), _p32(dst), n_nt, len(rules),
                        _p32(kind), _p32(lhs), _p32(x), _p32(y), len(want), _p32(out_nt),
                        _p64(bits) if bitmaps else None, _p64(counts), _p64(facts))
    if rc != 0:
        raise RuntimeError(f"oracle_cfl failed ({rc})")
    return {a: (int(counts[i]), bits[i] if bitmaps else None) for i, a in enumerate(want)}


def cfl_reach_rounds(n, src, lbl, dst, label_names, grammar, nonterminals=None, threads=1, bitmaps=True):
    """The relation of ``cfl_reach`` by semi-naive rounds over n x n bitsets
    (``oracle_cfl_rounds``): needs 3 n^2/8 bytes per normal-form nonterminal,
    but no per-fact joins, so it reaches larger graphs.  Returns
    ({name: (count, bitmap or None)}, rounds)."""
    lib = _load()
    label_ids = {name: i for i, name in enumerate(label_names)}
    n_nt, rules, names = lang.grammar_normal_form(grammar, label_ids)
    want = list(names) if nonterminals is None else list(nonterminals)
    out_nt = _u32([names.index(a) for a in want])
    src, lbl, dst = _u32(src), _u32(lbl), _u32(dst)
    kind = _u32([r[0] for r in rules])
    lhs = _u32([r[1] for r in rules])
    x = _u32([r[2] for r in rules])
    y = _u32([r[3] for r in rules])
    w = words(n)
    bits = np.zeros((len(want), n, w), dtype=np.uint64) if bitmaps else None
    counts = np.zeros(len(want), dtype=np.uint64)
    rounds = np.zeros(1, dtype=np.uint32)
    rc = lib.oracle_cfl_rounds(n, len(src), _p32(src), _p32(lbl), _p32(dst), n_nt, len(rules),
                               _p32(kind), _p32(lhs), _p32(x), _p32(y), len(want), _p32(out_nt),
                               _p64(bits) if bitmaps else None, _p64(counts), int(threads), _p32(rounds))
    if rc != 0:
        raise RuntimeError(f"oracle_cfl_rounds failed ({rc})")
    return {a: (int(counts[i]), bits[i] if bitmaps else None) for i, a in enumerate(want)}, int(rounds[0])


def pairs_hash(bm, n, row_ids=None, threads=1):
    """(count, hash) of the pairs of bitmap rows bm [rows, ceil(n/64)]: row i
    is vertex row_ids[i] (default i); hash = sum of splitmix64((u << 32) | v)
    mod 2^64 (SplitMix64 of Steele, Lea and Flood, 2014)."""
    lib = _load()
    bm = np.ascontiguousarray(bm, dtype=np.uint64)
    ids = None if row_ids is None else _u32(row_ids)
    c = np.zeros(1, dtype=np.uint64)
    h = np.zeros(1, dtype=np.uint64)
    lib.oracle_pairs_hash(n, bm.shape[0], _p32(ids) if ids is not None else None, _p64(bm), int(threads),
                          _p64(c), _p64(h))
    return int(c[0]), int(h[0])


def groups_hash(groups, threads=1):
    """(count, hash) of the union of G x G over disjoint vertex groups."""
    lib = _load()
    off = np.zeros(len(groups) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(g) for g in groups])
    members = _u32(np.concatenate([np.asarray(g, dtype=np.uint32) for g in groups]) if groups else [])
    c = np.zeros(1, dtype=np.uint64)
    h = np.zeros(1, dtype=np.uint64)
    lib.oracle_groups_hash(len(groups), _p64(off), _p32(members), int(threads), _p64(c), _p64(h))
    return int(c[0]), int(h[0])


def rpq_rows(n, src, lbl, dst, label_names, regex, sources, threads=1, return_visits=False):
    """Rows of the RPQ answer for the given source vertices (product BFS).

    Returns uint64 [len(sources), ceil(n/64)]: bit v of row i set iff some
    path sources[i]..v spells a word of the regex's language.
    """
    lib = _load()
    label_ids = {name: i for i, name in enumerate(label_names)}
    nq, moves, s, f = lang.regex_enfa(regex)
    # a symbol that is not a graph label can never be read: drop its moves
    kept = [(a, (EPS_LABEL if sym is None else label_ids[sym]), b)
            for a, sym, b in moves if sym is None or sym in label_ids]
    tsrc = _u32([m[0] for m in kept])
    tlbl = _u32([m[1] for m in kept])
    tdst = _u32([m[2] for m in kept])
    final = np.zeros(nq, dtype=np.uint8)
    final[f] = 1
    sources = _u32(sources)
    src, lbl, dst = _u32(src), _u32(lbl), _u32(dst)
    out = np.zeros((len(sources), words(n)), dtype=np.uint64)
    visits = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_rpq_rows(n, len(src), _p32(src), _p32(lbl), _p32(dst), max(1, len(label_names)),
                             nq, len(kept), _p32(tsrc), _p32(tlbl), _p32(tdst), s,
                             final.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(sources),
                             _p32(sources), _p64(out), int(threads), _p64(visits))
    if rc != 0:
        raise RuntimeError(f"oracle_rpq_rows failed ({rc})")
    return (out, int(visits[0])) if return_visits else out


def rpq_all(n, src, lbl, dst, label_names, regex, threads=1):
    """Full RPQ answer bitmap [n, ceil(n/64)] (every vertex as a source)."""
    return rpq_rows(n, src, lbl, dst, label_names, regex, np.arange(n, dtype=np.uint32), threads)


def bitmap_pairs(bm, n):
    """Sorted list of (u, v) pairs set in a row-major bitmap (small n only)."""
    bits = np.unpackbits(bm.view(np.uint8), axis=1, bitorder="little")[:, :n]
    us, vs = np.nonzero(bits)
    return list(zip(us.tolist(), vs.tolist()))
