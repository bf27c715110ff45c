"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

This module only draws random graphs and query texts.  It holds none of the
method's arithmetic and imports neither the product package nor the oracle.
Every generator takes an explicit seed and uses numpy's PCG64 generator, so a
(generator, parameters, seed) triple names one input exactly.

A graph is returned as a ``Graph`` tuple: vertex count, edge arrays
(src, label, dst) of dtype uint32, and the label names (label id = index).
Edges are a set: generators never emit duplicates.

The paper's own datasets (Tables 1 and 3) are not available; the shapes
below stand in for them, as described next to each generator.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

Graph = namedtuple("Graph", "n src lbl dst labels")

BASE_SEED = 210314688


def _dedupe(n, src, lbl, dst):
    key = (lbl.astype(np.uint64) * np.uint64(n) + src.astype(np.uint64)) * np.uint64(n) + dst.astype(np.uint64)
    _, idx = np.unique(key, return_index=True)
    idx.sort()
    return src[idx], lbl[idx], dst[idx]


def make_graph(n, edges, labels):
    """Build a Graph from an iterable of (src, label_name, dst) triples."""
    labels = list(labels)
    ids = {name: i for i, name in enumerate(labels)}
    if edges:
        s, l, d = zip(*[(u, ids[x], v) for u, x, v in edges])
    else:
        s, l, d = (), (), ()
    src = np.asarray(s, dtype=np.uint32)
    lbl = np.asarray(l, dtype=np.uint32)
    dst = np.asarray(d, dtype=np.uint32)
    src, lbl, dst = _dedupe(n, src, lbl, dst)
    return Graph(n, src, lbl, dst, labels)


def with_inverses(g, pairs):
    """Add an inverse label for each (label, inverse_label) name pair: every
    edge (u, x, v) gets (v, x_inverse, u) (the inverse relation of Sec. 4.2)."""
    labels = list(g.labels)
    src, lbl, dst = [g.src], [g.lbl], [g.dst]
    for name, inv in pairs:
        if inv not in labels:
            labels.append(inv)
        i, j = labels.index(name), labels.index(inv)
        sel = g.lbl == i
        src.append(g.dst[sel])
        dst.append(g.src[sel])
        lbl.append(np.full(int(sel.sum()), j, dtype=np.uint32))
    s, l, d = _dedupe(g.n, np.concatenate(src), np.concatenate(lbl), np.concatenate(dst))
    return Graph(g.n, s, l, d, labels)


# --------------------------------------------------------------------------
# paper example and closed-form families
# --------------------------------------------------------------------------

def paper_example():
    """The two-vertex graph of the paper's running example (Sec. 2.1 figure):
    0 -a-> 1, 1 -a-> 0, 1 -b-> 1."""
    return make_graph(2, [(0, "a", 1), (1, "a", 0), (1, "b", 1)], ["a", "b"])


def chain(word):
    """A simple path 0 -> 1 -> ... -> len(word) spelling the given labels."""
    labels = sorted(set(word))
    return make_graph(len(word) + 1, [(i, x, i + 1) for i, x in enumerate(word)], labels)


# --------------------------------------------------------------------------
# workload shapes
# --------------------------------------------------------------------------

def erdos_renyi(n, labels=("a", "b"), p=None, seed=BASE_SEED + 1):
    """Directed Erdos-Renyi graph: every ordered pair (u, v), u == v included,
    carries each label independently with probability p (default 2/n).
    Shape of the balanced-bracket workload (n = 256)."""
    rng = np.random.default_rng(seed)
    p = 2.0 / n if p is None else p
    src, lbl, dst = [], [], []
    for i, _ in enumerate(labels):
        m = rng.random((n, n)) < p
        u, v = np.nonzero(m)
        src.append(u.astype(np.uint32))
        dst.append(v.astype(np.uint32))
        lbl.append(np.full(len(u), i, dtype=np.uint32))
    return Graph(n, np.concatenate(src), np.concatenate(lbl), np.concatenate(dst), list(labels))


def zipf_probs(k, s=1.2):
    w = 1.0 / np.arange(1, k + 1) ** s
    return w / w.sum()


def _uniform_targets(rng, n, deg):
    """For each vertex u, deg[u] distinct targets drawn uniformly from V minus u."""
    m = int(deg.sum())
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = rng.integers(0, n - 1, size=m)
    dst = dst + (dst >= src)                      # skip u itself
    # resample duplicates within a row until every row's targets are distinct
    for _ in range(100):
        key = src * n + dst
        order = np.argsort(key, kind="stable")
        dup = np.zeros(m, dtype=bool)
        ks = key[order]
        dup[order[1:][ks[1:] == ks[:-1]]] = True
        if not dup.any():
            break
        k = int(dup.sum())
        nd = rng.integers(0, n - 1, size=k)
        dst[dup] = nd + (nd >= src[dup])
    return src.astype(np.uint32), dst.astype(np.uint32)


def powerlaw(n, labels=("a", "b", "c", "d"), mean_deg=4.0, alpha=2.1, zipf_s=1.2, seed=BASE_SEED + 2):
    """Power-law directed graph for regular path queries (stand-in for the RDF
    graphs of Table 1).  Out-degrees round(Pareto(alpha, x_m)) with x_m chosen
    so the mean is mean_deg, clipped to [1, n-1]; targets uniform without
    replacement, no self-loops; labels iid Zipf(zipf_s) over the label list."""
    rng = np.random.default_rng(seed)
    xm = mean_deg * (alpha - 1.0) / alpha
    deg = np.rint(xm * (1.0 + rng.pareto(alpha, size=n))).astype(np.int64)
    deg = np.clip(deg, 1, n - 1)
    src, dst = _uniform_targets(rng, n, deg)
    lbl = rng.choice(len(labels), size=len(src), p=zipf_probs(len(labels), zipf_s)).astype(np.uint32)
    return Graph(n, src, lbl, dst, list(labels))


def hierarchy(n, branching=4.0, type_frac=0.2, with_type=True, seed=BASE_SEED + 3):
    """Random tree plus 'type' edges (stand-in for the RDF class hierarchies of
    Table 3).  The tree grows level by level, each vertex taking Poisson(
    branching) children (a level's first vertex at least one) until n vertices
    exist; 'sc' edges point parent -> child.  A uniform sample of type_frac of
    the vertices gets one 'type' edge to a uniform other vertex.  Inverse
    labels 'sc_r' and 'type_r' are added.  Also returns the depth array."""
    rng = np.random.default_rng(seed)
    parent = np.full(n, -1, dtype=np.int64)
    depth = np.zeros(n, dtype=np.int64)
    nxt, level = 1, [0]
    while nxt < n:
        new_level = []
        for i, p in enumerate(level):
            k = int(rng.poisson(branching))
            if i == 0:
                k = max(k, 1)
            k = min(k, n - nxt)
            for _ in range(k):
                parent[nxt] = p
                depth[nxt] = depth[p] + 1
                new_level.append(nxt)
                nxt += 1
            if nxt >= n:
                break
        level = new_level
    child = np.arange(1, n)
    edges_s = [parent[1:].astype(np.uint32)]
    edges_d = [child.astype(np.uint32)]
    edges_l = [np.zeros(n - 1, dtype=np.uint32)]
    labels = ["sc", "type"]
    if with_type:
        k = int(round(type_frac * n))
        who = rng.choice(n, size=k, replace=False)
        to = rng.integers(0, n - 1, size=k)
        to = to + (to >= who)
        edges_s.append(who.astype(np.uint32))
        edges_d.append(to.astype(np.uint32))
        edges_l.append(np.ones(k, dtype=np.uint32))
    g = Graph(n, np.concatenate(edges_s), np.concatenate(edges_l), np.concatenate(edges_d), labels)
    g = with_inverses(g, [("sc", "sc_r"), ("type", "type_r")])
    return g, depth


def clustered(n, mean_deg=1.0, cluster=(64, 512), local=0.95, d_share=0.77, seed=BASE_SEED + 4):
    """Program-like graph for the alias query (stand-in for the Linux-kernel
    graphs of Table 3).  Vertices are cut into consecutive clusters with sizes
    uniform in [cluster]; n*mean_deg base edges, each with a uniform source and
    a target inside the source's cluster (other than the source) with
    probability local, else uniform; label 'd' with probability d_share else
    'a'; inverse labels 'a_r', 'd_r' are added, so the average degree counting
    both directions is 2*mean_deg."""
    rng = np.random.default_rng(seed)
    sizes = []
    total = 0
    while total < n:
        s = int(rng.integers(cluster[0], cluster[1] + 1))
        s = min(s, n - total)
        sizes.append(s)
        total += s
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    cid = np.repeat(np.arange(len(sizes)), sizes)
    m = int(round(n * mean_deg))
    src = rng.integers(0, n, size=m)
    lo, sz = starts[cid[src]], np.asarray(sizes)[cid[src]]
    loc = rng.random(m) < local
    t_local = lo + rng.integers(0, np.maximum(sz - 1, 1))
    t_local = t_local + (t_local >= src)
    t_local = np.where(sz > 1, t_local, src)
    t_glob = rng.integers(0, n, size=m)
    dst = np.where(loc, t_local, t_glob)
    lbl = np.where(rng.random(m) < d_share, 1, 0).astype(np.uint32)   # 0 = a, 1 = d
    s, l, d = _dedupe(n, src.astype(np.uint32), lbl, dst.astype(np.uint32))
    g = Graph(n, s, l, d, ["a", "d"])
    return with_inverses(g, [("a", "a_r"), ("d", "d_r")])


# --------------------------------------------------------------------------
# query texts (the paper's queries, Sec. 4.2, and the example of Sec. 2.3)
# --------------------------------------------------------------------------

BRACKETS = "S -> a S b | a b"
RPQ_C2 = "(a | b)* c d*"
SAME_GEN_G1 = "S -> sc_r S sc | type_r S type | sc_r sc | type_r type"
SAME_GEN_G2 = "S -> sc_r S sc | sc"
SAME_GEN_SC = "S -> sc_r S sc | sc_r sc"
MEM_ALIAS = "S -> d_r V d\nV -> ((S?) a_r)* (S?) (a (S?))*"


def random_regex(rng, labels, min_syms=2, max_syms=8):
    """A random regular expression over the given labels, shaped like the
    templates of Table 2: alternations, concatenations, star, plus, option."""
    target = int(rng.integers(min_syms, max_syms + 1))

    def gen(k):
        if k <= 1:
            return str(rng.choice(labels))
        r = rng.random()
        if r < 0.35:
            a = int(rng.integers(1, k))
            return f"({gen(a)} | {gen(k - a)})"
        if r < 0.75:
            a = int(rng.integers(1, k))
            return f"{gen(a)} {gen(k - a)}"
        return f"({gen(k)}){str(rng.choice(['*', '+', '?']))}"

    return gen(target)


def random_cfg(rng, labels, n_nt=(2, 6), eps_prob=0.05):
    """A random grammar in normal form (A -> B C | A -> t | rarely A -> eps)
    with 2..6 nonterminals whose start nonterminal derives some word
    (checked syntactically: productive-nonterminal fixpoint)."""
    while True:
        k = int(rng.integers(n_nt[0], n_nt[1] + 1))
        names = [f"N{i}" for i in range(k)]
        rules = {a: [] for a in names}
        for a in names:
            for _ in range(int(rng.integers(1, 4))):
                r = rng.random()
                if r < eps_prob:
                    rules[a].append("eps")
                elif r < 0.45:
                    rules[a].append(str(rng.choice(labels)))
                else:
                    rules[a].append(f"{rng.choice(names)} {rng.choice(names)}")
        productive, grew = set(), True
        while grew:
            grew = False
            for a in names:
                if a in productive:
                    continue
                for alt in rules[a]:
                    syms = alt.split()
                    if all(s == "eps" or s not in rules or s in productive for s in syms):
                        productive.add(a)
                        grew = True
                        break
        if names[0] in productive:
            return "\n".join(f"{a} -> {' | '.join(rules[a])}" for a in names)


def serving_mix(n_graphs=64, n_queries=10000, n_range=(1000, 200000), mean_deg=3.0, n_labels=8,
                seed=BASE_SEED + 5, graph_seed_stride=1000):
    """Graphs and query texts of the batched-serving workload: n_graphs graphs
    with n log-uniform in n_range and power-law out-degrees, 8 Zipf labels;
    n_queries queries, each on a uniformly chosen graph, half random regexes
    and half random small grammars over 4..8 of that graph's labels.
    Graphs are returned as (n, seed) recipes so callers build them lazily."""
    rng = np.random.default_rng(seed)
    labels = [f"l{i}" for i in range(n_labels)]
    ns = np.rint(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), size=n_graphs))).astype(int)
    graphs = [(int(ns[i]), seed + graph_seed_stride * (i + 1)) for i in range(n_graphs)]
    queries = []
    for q in range(n_queries):
        gi = int(rng.integers(0, n_graphs))
        k = int(rng.integers(4, n_labels + 1))
        use = [str(x) for x in rng.choice(labels, size=k, replace=False)]
        if rng.random() < 0.5:
            queries.append((gi, "regex", random_regex(rng, use)))
        else:
            queries.append((gi, "cfg", random_cfg(rng, use)))
    return labels, graphs, queries


def serving_graph(n, seed, labels, mean_deg=3.0):
    return powerlaw(n, labels=tuple(labels), mean_deg=mean_deg, seed=seed)


# (a|b)* c d* as a four-state automaton (a deterministic automaton that is
# not minimal: the states after c and after d accept the same words):
# 0 -a,b-> 1, 1 -a,b-> 1, 0 -c-> 2, 1 -c-> 2, 2 -d-> 3, 3 -d-> 3, final {2, 3}
RPQ_C2_FOUR_STATE = (4, [(0, "a", 1), (0, "b", 1), (1, "a", 1), (1, "b", 1), (0, "c", 2), (1, "c", 2),
                         (2, "d", 3), (3, "d", 3)], {2, 3})
