"""All paths of bounded length (Sec. 3.2, paths extraction) against brute
force.  Every path u -> v with at most L edges is listed from the graph
itself, and kept iff a recogniser written from the definition of a
derivation (tests/brute.py) accepts its word (grammars) or Python's re
matches it (regular queries).  The library must return exactly that set,
each path once, with non-decreasing lengths."""
import json
import re
from pathlib import Path

import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod
from tests import brute

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def graph_paths(edges, u, v, max_len):
    """Every edge sequence u -> v of at most max_len edges (the empty one if u == v)."""
    succ = {}
    for a, x, b in sorted(set(edges)):
        succ.setdefault(a, []).append((x, b))
    out = []

    def walk(node, path):
        if node == v:
            out.append(tuple(path))
        if len(path) == max_len:
            return
        for x, b in succ.get(node, ()):
            path.append((node, x, b))
            walk(b, path)
            path.pop()

    walk(u, [])
    return out


def library_paths(res, u, v, max_len, box=0):
    got = [tuple(map(tuple, p.tolist())) for p in res.paths(u, v, max_len, box=box)]
    lens = [len(p) for p in got]
    assert lens == sorted(lens), "lengths must not decrease"
    assert len(set(got)) == len(got), "a path was returned twice"
    return got


def labelled(g):
    return [(int(a), g.labels[int(x)], int(b)) for a, x, b in zip(g.src, g.lbl, g.dst)]


def run(g, text, kind, **kw):
    R = rsm_mod.from_regex(text, g.labels) if kind == "regex" else rsm_mod.from_grammar(text, g.labels)
    res = cfpq.query(cfpq.Graph.from_synth(g), cfpq.Query(R), keep_rank=True, **kw)
    return R, res


def check_all_pairs(g, accepts, res, max_len, pairs=None):
    named = labelled(g)
    ids = {e: (int(a), int(x), int(b)) for e, a, x, b in zip(named, g.src, g.lbl, g.dst)}
    cache = {}

    def ok(word):
        if word not in cache:
            cache[word] = accepts(word)
        return cache[word]

    total = 0
    for u, v in pairs or [(u, v) for u in range(g.n) for v in range(g.n)]:
        want = {tuple(ids[e] for e in p) for p in graph_paths(named, u, v, max_len) if ok(tuple(e[1] for e in p))}
        got = library_paths(res, u, v, max_len)
        assert set(got) == want, (u, v, sorted(want ^ set(got))[:4])
        total += len(got)
    return total


def random_graph(rng, n, labels, p):
    edges = [(u, str(rng.choice(labels)), v) for u in range(n) for v in range(n) if rng.random() < p]
    return synth.make_graph(n, edges, list(labels))


GRAMMARS = {
    "brackets": ([("S", ["a", "S", "b"]), ("S", ["a", "b"])], ["a", "b"]),
    "ambiguous": ([("S", ["S", "S"]), ("S", ["a"])], ["a"]),
    "left_rec_eps": ([("S", ["S", "a"]), ("S", [])], ["a", "b"]),
    "nullable_pair": ([("S", ["S", "S"]), ("S", ["a"]), ("S", ["b", "S", "c"]), ("S", [])], ["a", "b", "c"]),
    "two_boxes": ([("S", ["A", "b", "A"]), ("A", ["a", "A"]), ("A", [])], ["a", "b"]),
}


@pytest.mark.parametrize("name", sorted(GRAMMARS))
def test_grammar_paths_match_brute_force(name):
    prods, labels = GRAMMARS[name]
    rng = np.random.default_rng(sum(map(ord, name)))
    g = random_graph(rng, 5, labels, 0.3)
    R, res = run(g, brute.bnf_text(prods), "grammar")
    assert R.box_names[0] == prods[0][0]
    n = check_all_pairs(g, lambda w: brute.bnf_accepts(prods, prods[0][0], w), res, 6)
    assert n > 0


def test_random_grammars_paths_match_brute_force():
    rng = np.random.default_rng(synth.BASE_SEED + 71)
    done = 0
    for _ in range(40):
        terms = ["a", "b", "c"]
        k = int(rng.integers(1, 4))
        names = [f"N{i}" for i in range(k)]
        prods = []
        for a in names:
            for _ in range(int(rng.integers(1, 4))):
                ln = int(rng.choice([0, 1, 1, 2, 2, 2, 3]))
                prods.append((a, [str(rng.choice(names + terms)) for _ in range(ln)]))
        if names[0] not in {a for a, _ in prods}:
            continue
        g = random_graph(rng, 4, terms, 0.35)
        R, res = run(g, brute.bnf_text(prods), "grammar")
        check_all_pairs(g, lambda w: brute.bnf_accepts(prods, "N0", w), res, 5)
        done += 1
    assert done >= 20


@pytest.mark.parametrize("regex,py", [("(a | b)* c", "(a|b)*c"), ("a*", "a*"), ("a b* | c", "ab*|c"),
                                      ("(a b)+ c?", "(ab)+c?")])
def test_regex_paths_match_brute_force(regex, py):
    rng = np.random.default_rng(len(regex))
    g = random_graph(rng, 5, ["a", "b", "c"], 0.3)
    _, res = run(g, regex, "regex")
    pat = re.compile(py)
    check_all_pairs(g, lambda w: pat.fullmatch("".join(w)) is not None, res, 6)


def test_paper_example_paths():
    # the graph and grammar of the worked example (Sec. 3.3): S derives a^k b^k
    d = json.loads((Path(__file__).parent / "golden" / "paper_example.json").read_text())
    g = synth.make_graph(d["n"], [tuple(e) for e in d["edges"]], d["labels"])
    prods = [("S", ["a", "S", "b"]), ("S", ["a", "b"])]
    _, res = run(g, brute.bnf_text(prods), "grammar")
    for L in (2, 5, 8):
        check_all_pairs(g, lambda w: brute.bnf_accepts(prods, "S", w), res, L)
    # 0 -> 1: a b, then a^3 b^3 (0 has no b edge, so a^2 b^2 cannot start there);
    # 1 -> 1: a^2 b^2 round the cycle first
    assert [len(p) for p in library_paths(res, 0, 1, 6)] == [2, 6]
    assert [len(p) for p in library_paths(res, 1, 1, 4)] == [4]


def test_bound_zero_and_empty_path():
    g = synth.make_graph(3, [(0, "a", 1), (1, "a", 2)], ["a"])
    _, res = run(g, "a*", "regex")
    assert library_paths(res, 1, 1, 0) == [()]
    assert library_paths(res, 0, 2, 1) == []
    assert library_paths(res, 0, 2, 2) == [((0, 0, 1), (1, 0, 2))]


def test_masked_pair_has_no_paths_and_buffer_protocol():
    g = synth.make_graph(4, [(0, "a", 1), (1, "a", 2), (2, "a", 3), (3, "a", 0)], ["a"])
    R = rsm_mod.from_regex("a+", g.labels)
    graph = cfpq.Graph.from_synth(g)
    src = np.array([True, False, False, False])
    res = cfpq.query(graph, cfpq.Query(R), keep_rank=True, src_mask=src)
    assert library_paths(res, 1, 2, 8) == []
    assert [len(p) for p in library_paths(res, 0, 2, 10)] == [2, 6, 10]
    # too small a buffer: the path is kept for the next call
    it = cfpq.cfpq_paths_open(res.h, 0, 0, 2, 10)
    try:
        lib = cfpq.load()
        import ctypes
        n = ctypes.c_uint64()
        assert lib.cfpq_paths_next(it, None, 0, ctypes.byref(n)) == cfpq.ERR_BUFFER and n.value == 2
        p = cfpq.cfpq_paths_next(it, cap=2)
        assert p.tolist() == [[0, 0, 1], [1, 0, 2]]
    finally:
        cfpq.cfpq_paths_close(it)


def test_paths_without_ranks_and_valid_arguments():
    g = synth.make_graph(3, [(0, "a", 1)], ["a"])
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_regex("a", g.labels))
    res = cfpq.query(graph, q)          # no ranks: all paths need only the index
    assert library_paths(res, 0, 1, 3) == [((0, 0, 1),)]
    for args in [(1, 0, 1, 3), (0, 3, 1, 3), (0, 0, 9, 3)]:
        with pytest.raises(cfpq.CfpqError) as e:
            cfpq.cfpq_paths_open(res.h, *args)
        assert e.value.status == cfpq.ERR_INVALID


def test_larger_graph_paths_sampled():
    # a same-generation graph: paths of G1 up to 6 edges for sampled pairs,
    # against brute force restricted to those pairs
    g, _ = synth.hierarchy(60, seed=72)
    prods = [("S", ["sc_r", "S", "sc"]), ("S", ["type_r", "S", "type"]), ("S", ["sc_r", "sc"]),
             ("S", ["type_r", "type"])]
    _, res = run(g, brute.bnf_text(prods), "grammar")
    pairs = [(int(u), int(v)) for u, v in res.pairs(0)[:: max(1, len(res.pairs(0)) // 12)].tolist()]
    n = check_all_pairs(g, lambda w: brute.bnf_accepts(prods, "S", w), res, 6, pairs=pairs)
    assert n >= len(pairs)


# ---------------------------------------------------------------------------
# witnesses and bounded paths at the workloads' sizes (validity checks: the
# edges exist and join up, the word is in the language)
# ---------------------------------------------------------------------------
def _valid(path, u, v, edges, accepts, labels):
    if len(path) == 0:
        return u == v
    assert path[0][0] == u and path[-1][2] == v
    for (a, _, b), (c, _, d) in zip(path, path[1:]):
        assert b == c
    assert all((int(x), int(lb), int(y)) in edges for x, lb, y in path)
    return accepts(tuple(labels[int(lb)] for _, lb, _ in path))


def test_rpq_witnesses_and_paths_at_bench_size():
    print("paths: RPQ witnesses and paths, power-law n=100000, no ranks kept", flush=True)
    g = synth.powerlaw(100000, seed=synth.BASE_SEED + 2)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels)
    graph, q = cfpq.Graph.from_synth(g), cfpq.Query(R)
    res = cfpq.query(graph, q)
    edges = set(zip(g.src.tolist(), g.lbl.tolist(), g.dst.tolist()))
    pat = re.compile("(a|b)*cd*")
    accepts = lambda w: pat.fullmatch("".join(w)) is not None
    bm = res.bitmap(0)
    rng = np.random.default_rng(91)
    checked = 0
    for u in rng.choice(g.n, size=12, replace=False).tolist():
        row = np.unpackbits(bm[u].view(np.uint8), bitorder="little")[:g.n]
        vs = np.flatnonzero(row)
        if not len(vs):
            continue
        for v in rng.choice(vs, size=min(3, len(vs)), replace=False).tolist():
            path = res.extract_path(u, v)
            assert _valid(path, u, v, edges, accepts, g.labels)
            # all paths of at most 4 edges: every one valid, shortest first,
            # and the witness's length is the least one when it is within 4
            ps = library_paths(res, u, v, 4)
            assert all(_valid(np.asarray(p), u, v, edges, accepts, g.labels) for p in ps if p)
            if len(path) <= 4:
                assert ps and len(ps[0]) <= len(path)
            checked += 1
    assert checked >= 10
    # a pair outside the relation
    u = int(np.flatnonzero(bm.sum(axis=1) == 0)[0]) if (bm.sum(axis=1) == 0).any() else None
    if u is not None:
        with pytest.raises(cfpq.CfpqError) as e:
            res.extract_path(u, (u + 1) % g.n)
        assert e.value.status == cfpq.ERR_NOT_FOUND


def test_grammar_witnesses_and_paths_at_samegen_size():
    print("paths: same-generation witnesses and paths, hierarchy n=50000, ranks kept on the device", flush=True)
    g, _ = synth.hierarchy(50000, seed=synth.BASE_SEED + 3)
    prods = [("S", ["sc_r", "S", "sc"]), ("S", ["type_r", "S", "type"]), ("S", ["sc_r", "sc"]),
             ("S", ["type_r", "type"])]
    R = rsm_mod.from_grammar(synth.SAME_GEN_G1, g.labels)
    res = cfpq.query(cfpq.Graph.from_synth(g), cfpq.Query(R), keep_rank=True)
    edges = set(zip(g.src.tolist(), g.lbl.tolist(), g.dst.tolist()))
    accepts = lambda w: brute.bnf_accepts(prods, "S", w)
    rng = np.random.default_rng(92)
    bm = res.bitmap(0)
    rows = np.flatnonzero(bm.any(axis=1))
    checked = 0
    for u in rng.choice(rows, size=10, replace=False).tolist():
        vs = np.flatnonzero(np.unpackbits(bm[u].view(np.uint8), bitorder="little")[:g.n])
        for v in rng.choice(vs, size=min(2, len(vs)), replace=False).tolist():
            path = res.extract_path(u, v)
            assert _valid(path, u, v, edges, accepts, g.labels)
            # bounded paths: the iterator memoises one n-bit set per
            # (symbol, vertex, length) it visits, so the bound is kept short here
            L = min(8, len(path) + 2)
            ps = library_paths(res, u, v, L)
            assert all(_valid(np.asarray(p), u, v, edges, accepts, g.labels) for p in ps)
            if len(path) <= L:
                assert ps and len(ps[0]) <= len(path)
            checked += 1
    assert checked >= 10
