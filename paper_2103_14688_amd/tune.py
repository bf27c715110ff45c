"""Autotuner: picks, per class of query, the closure strategy, the
nonterminal-product mode, the source-tile width and the closure arm
(incremental, Sec. 3.1.1, or recomputed from scratch each iteration, the
variant the paper measured) from measurements, and keeps them in a JSON cache
on disk.

A query's class is a key of measured features that decide which variant
wins: the size class of the graph (log2 n), its mean degree class, the
number of RSM states and boxes, whether the query has box-labelled
transitions (a grammar) or not (a regular query, one productive iteration),
and whether some box is nullable.  The candidates include the literal
per-edge closure for small classes.  The first query of a class runs every
candidate once (each a complete, correct query: the answer does not depend
on the choice) and records the fastest; later queries of the class run the
recorded choice.  Within a query the library switches formats by itself:
per source row, sparse lists (ELL) for rows of at most 32 bits in the tile
and the LDS-blocked dense product for denser rows, every closure level anew.

Only arguments of the C ABI are chosen here; all computation stays in the
HIP library.
"""
from __future__ import annotations

import json
import math
import os
import threading
import time

from . import cfpq

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "cfpq_gfx950", "tune.json")
PEREDGE_MAX_NODES = 4096   # product nodes (upper bound from the class key) for the per-edge arm


def features(graph, rsm):
    """Class key of a (graph, RSM) pair."""
    n, _, m = graph.info()
    has_calls = bool((rsm.t_sym >= rsm.n_terminals).any()) if len(rsm.t_sym) else False
    nullable = bool(any(rsm.is_final[int(s)] for s in rsm.box_start))
    deg = m / max(1, n)
    return {
        "n_log2": int(math.floor(math.log2(max(1, n)))),
        "deg_class": int(math.floor(math.log2(max(1.0, deg)))),
        "states": int(rsm.n_states),
        "boxes": int(rsm.n_boxes),
        "grammar": has_calls,
        "nullable": nullable,
    }


def key_of(feat):
    return "n{n_log2}-d{deg_class}-q{states}-b{boxes}-{g}{e}".format(
        g="cfg" if feat["grammar"] else "rpq", e="-eps" if feat["nullable"] else "", **feat)


def candidates(feat):
    """Option sets worth measuring for a class (each a dict of cfpq.query
    keyword arguments)."""
    small = feat["n_log2"] <= 10 and feat["boxes"] <= 64   # n < 2048: the fused kernel applies
    out = []
    if small:
        out.append({"strategy": cfpq.STRATEGY_FUSED})
    # the literal per-edge closure (Sec. 3.1.1) as an arm of its own where it
    # finishes in well under a second (states * n up to 4096; its limit is
    # 65536); it has never been the fastest, but the tuner measures, not assumes
    if feat["states"] * (2 << feat["n_log2"]) <= PEREDGE_MAX_NODES:
        out.append({"strategy": cfpq.STRATEGY_PEREDGE})
    if not feat["grammar"]:
        out.append({"strategy": cfpq.STRATEGY_CONDENSED})
        out.append({"strategy": cfpq.STRATEGY_LEVELS})
        return out
    words = (1 << feat["n_log2"]) // 64 + 1
    out.append({"strategy": cfpq.STRATEGY_LEVELS, "nt_mode": cfpq.NT_AUTO, "tile_words": 0})
    out.append({"strategy": cfpq.STRATEGY_LEVELS, "nt_mode": cfpq.NT_ROWS, "tile_words": 0})
    if words > 1200:
        # untiled (one tile per query) against the automatic cap
        out.append({"strategy": cfpq.STRATEGY_LEVELS, "nt_mode": cfpq.NT_AUTO, "tile_words": min(words, 4096)})
    out.append({"strategy": cfpq.STRATEGY_LEVELS, "nt_mode": cfpq.NT_AUTO, "tile_words": 0, "recompute": True})
    return out


class Tuner:
    """Measured choices per query class, persisted as JSON at `path`."""

    def __init__(self, path=DEFAULT_CACHE, runs=1):
        self.path = path
        self.runs = runs
        self.lock = threading.Lock()
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def save(self):
        if not self.path:
            return
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    @staticmethod
    def _time(graph, q, opts, runs):
        best = None
        for _ in range(runs):
            t = time.perf_counter()
            r = cfpq.query(graph, q, **opts)
            r.stats()     # the call returns after the fixpoint; stats are host-side
            dt = time.perf_counter() - t
            r.close()
            best = dt if best is None else min(best, dt)
        return best

    def tune(self, graph, q, force=False):
        """The recorded choice for q's class, measuring every candidate first
        if the class is new (or force).  Returns (options, entry)."""
        feat = features(graph, q.rsm)
        key = key_of(feat)
        with self.lock:
            if key in self.table and not force:
                e = self.table[key]
                return dict(e["options"]), e
        measured = []
        for opts in candidates(feat):
            try:
                ms = self._time(graph, q, opts, self.runs) * 1e3
            except cfpq.CfpqError as err:      # e.g. out of memory for an untiled choice
                measured.append({"options": opts, "ms": None, "error": str(err)})
                continue
            measured.append({"options": opts, "ms": ms})
        ok = [m for m in measured if m["ms"] is not None]
        if not ok:
            raise RuntimeError(f"no candidate ran for class {key}")
        best = min(ok, key=lambda m: m["ms"])
        entry = {"features": feat, "options": best["options"], "ms": best["ms"], "measured": measured}
        with self.lock:
            self.table[key] = entry
            self.save()
        return dict(best["options"]), entry

    def query(self, graph, q, **kw):
        """cfpq.query with the class's recorded (or newly measured) choice;
        kw (masks, stream, keep_rank, ...) pass through."""
        opts, _ = self.tune(graph, q)
        opts.update(kw)
        return cfpq.query(graph, q, **opts)
