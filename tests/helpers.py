"""Shared test helpers: run a query through the C ABI and compute the oracle's
answer for the same seeded input."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2103_14688_amd import rsm as rsm_mod

MASK64 = (1 << 64) - 1


def splitmix64_np(x):
    """SplitMix64 first output for seeds x (uint64 array), wrapping arithmetic."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def bitmap_hash(bm, n):
    """Order-independent pair hash of a row-major bitmap (sum of splitmix64)."""
    bits = np.unpackbits(bm.view(np.uint8), axis=1, bitorder="little")[:, :n]
    u, v = np.nonzero(bits)
    keys = (u.astype(np.uint64) << np.uint64(32)) | v.astype(np.uint64)
    with np.errstate(over="ignore"):
        return int(splitmix64_np(keys).sum(dtype=np.uint64))


def popcount(bm):
    return int(np.unpackbits(bm.view(np.uint8)).sum())


def oracle_grammar(g, text, names=None):
    return oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, text, names)


def oracle_regex(g, text, threads=8):
    return oracle.rpq_all(g.n, g.src, g.lbl, g.dst, g.labels, text, threads=threads)


def compile_query(kind, text, labels, minimize=True):
    if kind == "regex":
        return rsm_mod.from_regex(text, labels, minimize)
    return rsm_mod.from_grammar(text, labels, minimize)


def bits_to_pairs(bm, n):
    bits = np.unpackbits(bm.view(np.uint8), axis=1, bitorder="little")[:, :n]
    return set(zip(*[a.tolist() for a in np.nonzero(bits)]))


def padding_clear(bm, n):
    """Bits at columns >= n must be zero."""
    if n % 64 == 0:
        return True
    last = bm[:, -1]
    mask = np.uint64(~((1 << (n % 64)) - 1) & MASK64)
    return not np.any(last & mask)
