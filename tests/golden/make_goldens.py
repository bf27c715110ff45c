"""Writes tests/golden/fullsize.json: pair counts and order-independent
hashes of the relations of the measured workloads at their full sizes.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
inputs of ``synth/``; nothing from the product package is imported.  The
hash of a pair set is the sum of splitmix64((u << 32) | v) modulo 2^64
(SplitMix64 of Steele, Lea and Flood, 2014), so a relation too large to store
is compared by (count, hash).

  rpq_powerlaw_n100000     (a|b)* c d* on the power-law graph n = 100,000:
                           product-automaton BFS from every source, in
                           blocks of sources; also per-block values.
  samegen_g1_n50000        same-generation G1 on the hierarchy graph
                           n = 50,000 with type edges: semi-naive rounds.
  samegen_g2_n50000        same-generation G2, same graph.
  samegen_typefree_n200000 G1 on the hierarchy n = 200,000 without type
                           edges: the closed form (all pairs of vertices of
                           equal depth >= 1; Sec. 4.2 query on a tree),
                           counted and hashed group by group.
  samegen_typefree_n500000 the same at n = 500,000 (the largest hierarchy).
  alias_n20000             memory alias MA on the clustered graph
                           n = 20,000 (clusters of 64..512 vertices):
                           semi-naive rounds; both nonterminals.
  serving                  the serving mix (64 graphs, n log-uniform in
                           [1e3, 2e5], 10,000 queries): every query on a graph
                           of at most 16,000 vertices, through the semi-naive
                           rounds (a regular query as the one-rule grammar
                           S -> regex) -> "full"; and a seeded 2% sample of
                           the others: regular queries on 64 seeded source
                           rows (BFS) -> "rows", grammars in full where
                           n <= 25,000 -> "full", the rest -> "unpinned".

Usage: python tests/golden/make_goldens.py [--only key,key] [--threads N]
Existing keys not asked for are kept.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")
SERVING_SMALL_N = 16000
SERVING_SAMPLE = 0.02
SERVING_SAMPLE_ROWS = 64
SERVING_GRAMMAR_MAX_N = 25000


def _hex(h):
    return f"{h:016x}"


def rpq_powerlaw(threads):
    n = 100000
    g = synth.powerlaw(n, seed=synth.BASE_SEED + 2)
    block = 5000
    total_c, total_h, blocks = 0, 0, []
    t = time.time()
    for b0 in range(0, n, block):
        srcs = np.arange(b0, min(n, b0 + block), dtype=np.uint32)
        rows = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=threads)
        c, h = oracle.pairs_hash(rows, g.n, row_ids=srcs, threads=threads)
        blocks.append({"first_source": b0, "count": c, "hash": _hex(h)})
        total_c += c
        total_h = (total_h + h) % (1 << 64)
        print(f"  rpq block {b0}: {c} pairs", flush=True)
    return {"graph": "synth.powerlaw(100000, seed=BASE_SEED + 2)", "query": synth.RPQ_C2, "box": "S",
            "count": total_c, "hash": _hex(total_h), "block_sources": block, "blocks": blocks,
            "oracle": "rpq_rows (product-automaton BFS per source)", "seconds": round(time.time() - t, 1)}


def _grammar_entry(g, text, recipe, threads, names=None):
    t = time.time()
    rel, nr = oracle.cfl_reach_rounds(g.n, g.src, g.lbl, g.dst, g.labels, text, names, threads=threads)
    out = {"graph": recipe, "query": text, "rounds": nr, "oracle": "cfl_reach_rounds (semi-naive rounds)",
           "boxes": {}}
    for a, (c, bm) in rel.items():
        c2, h = oracle.pairs_hash(bm, g.n, threads=threads)
        assert c2 == c
        out["boxes"][a] = {"count": c, "hash": _hex(h)}
    out["seconds"] = round(time.time() - t, 1)
    return out


def samegen(threads, which):
    n = 50000
    g, _ = synth.hierarchy(n, seed=synth.BASE_SEED + 3)
    text = synth.SAME_GEN_G1 if which == "g1" else synth.SAME_GEN_G2
    return _grammar_entry(g, text, "synth.hierarchy(50000, seed=BASE_SEED + 3)", threads)


def samegen_typefree(threads, n=200000):
    g, depth = synth.hierarchy(n, with_type=False, seed=synth.BASE_SEED + 3)
    groups = [np.flatnonzero(depth == d).astype(np.uint32) for d in range(1, int(depth.max()) + 1)]
    t = time.time()
    c, h = oracle.groups_hash(groups, threads=threads)
    return {"graph": f"synth.hierarchy({n}, with_type=False, seed=BASE_SEED + 3)", "query": synth.SAME_GEN_G1,
            "boxes": {"S": {"count": c, "hash": _hex(h)}},
            "oracle": "closed form: pairs of vertices of equal depth >= 1 (groups_hash)",
            "levels": [len(x) for x in groups], "seconds": round(time.time() - t, 1)}


def alias(threads):
    n = 20000
    g = synth.clustered(n, seed=synth.BASE_SEED + 4)
    return _grammar_entry(g, synth.MEM_ALIAS, "synth.clustered(20000, seed=BASE_SEED + 4)", threads)


def _serving_task(task):
    """One graph's share of the serving goldens: [(query id, entry)]."""
    gi, ids, threads = task
    labels, recipes, qs = synth.serving_mix()
    n, seed = recipes[gi]
    g = synth.serving_graph(n, seed, labels)
    out = []
    for i in ids:
        _, kind, text = qs[i]
        grammar = text if kind == "cfg" else f"S -> {text}"
        start = grammar.split("->", 1)[0].strip()
        if n <= SERVING_SMALL_N or (kind == "cfg" and n <= SERVING_GRAMMAR_MAX_N):
            rel, _ = oracle.cfl_reach_rounds(g.n, g.src, g.lbl, g.dst, g.labels, grammar, [start], threads=threads)
            c, h = oracle.pairs_hash(rel[start][1], g.n, threads=threads)
            out.append((i, [c, _hex(h)]))
        elif kind == "regex":
            srcs = _sample_rows(i, n)
            rows = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, text, srcs, threads=threads)
            c, h = oracle.pairs_hash(rows, g.n, row_ids=srcs, threads=threads)
            out.append((i, {"rows": srcs.tolist(), "count": c, "hash": _hex(h)}))
        else:
            out.append((i, None))
    return out


def _sample_rows(i, n):
    srng = np.random.default_rng(synth.BASE_SEED + 13 + i)
    return np.sort(srng.choice(n, size=SERVING_SAMPLE_ROWS, replace=False)).astype(np.uint32)


def serving(threads):
    import multiprocessing as mp

    labels, recipes, qs = synth.serving_mix()
    rng = np.random.default_rng(synth.BASE_SEED + 12)
    big = [i for i, (gi, _, _) in enumerate(qs) if recipes[gi][0] > SERVING_SMALL_N]
    sample = set(rng.choice(big, size=int(round(SERVING_SAMPLE * len(big))), replace=False).tolist())
    todo = [i for i, (gi, _, _) in enumerate(qs) if recipes[gi][0] <= SERVING_SMALL_N or i in sample]
    by_graph = {}
    for i in todo:
        by_graph.setdefault(qs[i][0], []).append(i)
    # tasks of at most 16 queries of one graph; the semi-naive rounds hold
    # 3 n^2/8 bytes per normal-form nonterminal (up to ~90 for these
    # grammars), so graphs are taken in three phases of fewer, wider
    # processes as n grows
    phases = [(0, 8000, threads, 1), (8000, SERVING_SMALL_N, max(1, min(3, threads)), 1),
              (SERVING_SMALL_N, 1 << 31, 1, threads)]
    out = {"mix": "synth.serving_mix()", "small_n": SERVING_SMALL_N, "sample_fraction": SERVING_SAMPLE,
           "sample_rows": SERVING_SAMPLE_ROWS, "grammar_max_n": SERVING_GRAMMAR_MAX_N,
           "full": {}, "rows": {}, "unpinned": []}
    t = time.time()
    for lo, hi, procs, th in phases:
        tasks = []
        for gi in sorted(by_graph, key=lambda x: recipes[x][0]):
            if lo < recipes[gi][0] <= hi:
                ids = by_graph[gi]
                tasks += [(gi, ids[j:j + 16], th) for j in range(0, len(ids), 16)]
        done = 0
        with mp.get_context("fork").Pool(procs) as pool:
            for res in pool.imap_unordered(_serving_task, tasks):
                for i, e in res:
                    if e is None:
                        out["unpinned"].append(i)
                    elif isinstance(e, dict):
                        out["rows"][str(i)] = e
                    else:
                        out["full"][str(i)] = e
                done += 1
                print(f"  serving n in ({lo}, {hi}]: task {done}/{len(tasks)} ({time.time() - t:.0f} s)", flush=True)
    out["unpinned"].sort()
    out["seconds"] = round(time.time() - t, 1)
    return out


JOBS = {
    "rpq_powerlaw_n100000": rpq_powerlaw,
    "samegen_g1_n50000": lambda th: samegen(th, "g1"),
    "samegen_g2_n50000": lambda th: samegen(th, "g2"),
    "samegen_typefree_n200000": samegen_typefree,
    "samegen_typefree_n500000": lambda th: samegen_typefree(th, 500000),
    "alias_n20000": alias,
    "serving": serving,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    oracle.build(force=False)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    keys = [k for k in args.only.split(",") if k] or list(JOBS)
    for k in keys:
        print(f"{k} ...", flush=True)
        data[k] = JOBS[k](args.threads)
        data[k]["generated_by"] = "tests/golden/make_goldens.py"
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(f"{k}: done in {data[k].get('seconds')} s", flush=True)


if __name__ == "__main__":
    main()
