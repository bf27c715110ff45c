"""Pins for the CPU oracle: values fixed by the paper and by mathematics,
not by the oracle itself.

* the paper's worked example (Sec. 3.3), from tests/golden/paper_example.json;
* closed forms: a^k b^k and (ab)^k chains for S -> a S b | a b (the language
  {a^n b^n, n > 0} of Sec. 2.3); same-depth pairs on a tree for the
  same-generation query (Sec. 4.2, G1 without type edges);
* library special cases: S -> a b is the Boolean product of the label
  matrices; (a|b)+ is the transitive closure of the union graph;
* brute force on tiny graphs: every path up to a length bound, word
  membership decided by an independent recogniser (grammar) or by Python's
  re module (regex); plus a naive relational fixpoint as a second,
  differently written evaluation of the same definition;
* invariants: the paper's symmetric queries give symmetric relations on
  graphs with inverse edges (Sec. 4.2), and an EBNF rule equals its
  hand-expanded BNF form.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import oracle
import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairs_of(bm, n):
    return set(oracle.bitmap_pairs(bm, n))


def edge_triples(g):
    return [(int(u), g.labels[int(x)], int(v)) for u, x, v in zip(g.src, g.lbl, g.dst)]


def test_paper_example():
    fx = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    g = synth.make_graph(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, fx["grammar"])
    assert pairs_of(r["S"][1], g.n) == {tuple(p) for p in fx["S"]}
    assert r["S"][0] == len(fx["S"])


def test_paper_example_witnesses_are_words_of_the_language():
    fx = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    prods = [("S", ["a", "S", "b"]), ("S", ["a", "b"])]
    edges = {tuple(e) for e in fx["edges"]}
    for key, path in fx["witnesses"].items():
        u, v = map(int, key.split(","))
        assert path[0][0] == u and path[-1][2] == v
        for (a, _, b), (c, _, d) in zip(path, path[1:]):
            assert b == c
        assert all(tuple(e) in edges for e in path)
        assert brute.bnf_accepts(prods, "S", tuple(e[1] for e in path))


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13])
def test_chain_anbn(k):
    g = synth.chain("a" * k + "b" * k)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.BRACKETS)
    assert pairs_of(r["S"][1], g.n) == {(k - j, k + j) for j in range(1, k + 1)}


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_chain_abab(k):
    g = synth.chain("ab" * k)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.BRACKETS)
    assert pairs_of(r["S"][1], g.n) == {(2 * i, 2 * i + 2) for i in range(k)}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_same_generation_closed_form(seed):
    g, depth = synth.hierarchy(600, with_type=False, seed=seed)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.SAME_GEN_SC)
    got = r["S"][1]
    d = depth
    want = (d[:, None] == d[None, :]) & (d[:, None] >= 1)
    bits = np.unpackbits(got.view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, want)
    levels = np.bincount(d)
    assert r["S"][0] == int((levels[1:] ** 2).sum())


def _dense(g, name):
    i = g.labels.index(name)
    sel = g.lbl == i
    return sp.csr_matrix((np.ones(int(sel.sum()), dtype=np.int64), (g.src[sel], g.dst[sel])), shape=(g.n, g.n))


@pytest.mark.parametrize("seed", [3, 4])
def test_concatenation_is_boolean_product(seed):
    g = synth.erdos_renyi(120, labels=("a", "b"), p=0.03, seed=seed)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, "S -> a b")
    prod = (_dense(g, "a") @ _dense(g, "b")).toarray() > 0
    bits = np.unpackbits(r["S"][1].view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, prod)


@pytest.mark.parametrize("seed", [5, 6])
def test_plus_is_transitive_closure(seed):
    g = synth.powerlaw(300, labels=("a", "b", "c"), mean_deg=1.5, seed=seed)
    union = (_dense(g, "a") + _dense(g, "b")).tocsr()
    want = np.zeros((g.n, g.n), dtype=bool)
    for u in range(g.n):
        # vertices reachable by >= 1 edge: BFS from u's successors
        succ = union.indices[union.indptr[u]:union.indptr[u + 1]]
        for s in succ:
            order = breadth_first_order(union, int(s), directed=True, return_predecessors=False)
            want[u, order] = True
    rows = oracle.rpq_all(g.n, g.src, g.lbl, g.dst, g.labels, "(a | b)+")
    bits = np.unpackbits(rows.view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, want)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, "S -> (a | b)+")
    assert np.array_equal(r["S"][1], rows)


def _random_bnf(rng, terms, k):
    names = [f"N{i}" for i in range(k)]
    prods = []
    for a in names:
        for _ in range(int(rng.integers(1, 4))):
            ln = int(rng.choice([0, 1, 1, 2, 2, 2, 3]))
            prods.append((a, [str(rng.choice(names + terms)) for _ in range(ln)]))
    return prods


def _tiny_graph(rng, n, labels, m):
    edges = {(int(rng.integers(0, n)), str(rng.choice(labels)), int(rng.integers(0, n))) for _ in range(m)}
    return sorted(edges)


@pytest.mark.parametrize("seed", range(40))
def test_grammar_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    labels = ["a", "b", "c"][: int(rng.integers(1, 4))]
    n = int(rng.integers(1, 4))
    edges = _tiny_graph(rng, n, labels, int(rng.integers(0, 6)))
    prods = _random_bnf(rng, labels, int(rng.integers(1, 4)))
    text = brute.bnf_text(prods)
    g = synth.make_graph(n, edges, labels)
    r = oracle.cfl_reach(n, g.src, g.lbl, g.dst, labels, text)
    naive = brute.relational_fixpoint(n, edges, prods)
    for a in {p[0] for p in prods}:
        got = pairs_of(r[a][1], n)
        assert got == naive[a], (text, edges, a)
    start = prods[0][0]
    found = brute.brute_cfl(n, edges, prods, start, 6)
    assert found <= pairs_of(r[start][1], n)


@pytest.mark.parametrize("seed", range(6))
def test_paper_grammars_brute_force(seed):
    rng = np.random.default_rng(2000 + seed)
    cases = [
        ([("S", ["a", "S", "b"]), ("S", ["a", "b"])], ["a", "b"]),
        ([("S", ["sc_r", "S", "sc"]), ("S", ["type_r", "S", "type"]), ("S", ["sc_r", "sc"]),
          ("S", ["type_r", "type"])], ["sc", "sc_r", "type", "type_r"]),
        ([("S", ["sc_r", "S", "sc"]), ("S", ["sc"])], ["sc", "sc_r"]),
    ]
    for prods, labels in cases:
        n = 4
        edges = _tiny_graph(rng, n, labels, 7)
        text = brute.bnf_text(prods)
        g = synth.make_graph(n, edges, labels)
        r = oracle.cfl_reach(n, g.src, g.lbl, g.dst, labels, text)
        got = pairs_of(r["S"][1], n)
        assert got == brute.relational_fixpoint(n, edges, prods)["S"]
        assert brute.brute_cfl(n, edges, prods, "S", 7) <= got


REGEXES = ["a", "a b*", "(a | b)* c d*", "a? b*", "(a b)+ | (c d)+", "a b (c | d | e)",
           "(a | b)+ (c | d)+", "(a (b c)*)+ | d e", "eps", "a*", "(a | eps) b"]


def _occurrences(regex):
    return len([t for t in regex.replace("(", " ").replace(")", " ").replace("|", " ").split()
                if t.strip("*+?") not in ("", "eps")])


@pytest.mark.parametrize("regex", REGEXES)
@pytest.mark.parametrize("seed", range(4))
def test_regex_brute_force(regex, seed):
    rng = np.random.default_rng(3000 + seed)
    labels = ["a", "b", "c", "d", "e"]
    occ = _occurrences(regex)
    n = 3 if occ <= 3 else 2
    # a shortest accepting path visits each (vertex, position-automaton state)
    # at most once, so its length is below (occurrences + 1) * n: brute force
    # up to that bound is exact
    bound = (occ + 1) * n
    assert bound <= 12
    edges = _tiny_graph(rng, n, labels, 6 if n == 3 else 5)
    g = synth.make_graph(n, edges, labels)
    rows = oracle.rpq_all(n, g.src, g.lbl, g.dst, labels, regex)
    got = pairs_of(rows, n)
    assert got == brute.brute_rpq(n, edges, regex, labels, bound)
    # the same query as a one-rule grammar through the worklist
    r = oracle.cfl_reach(n, g.src, g.lbl, g.dst, labels, f"S -> {regex}")
    assert pairs_of(r["S"][1], n) == got


@pytest.mark.parametrize("seed", [7, 8])
def test_same_generation_symmetric(seed):
    g, _ = synth.hierarchy(400, seed=seed)
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.SAME_GEN_G1)
    bits = np.unpackbits(r["S"][1].view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, bits.T)


def test_memory_alias_ebnf_equals_bnf_and_is_symmetric():
    g = synth.clustered(700, mean_deg=1.0, cluster=(8, 24), seed=9)
    bnf = "\n".join([
        "S -> d_r V d",
        "V -> L O R",
        "O -> S | eps",
        "L -> L O a_r | eps",
        "R -> a O R | eps",
    ])
    r1 = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.MEM_ALIAS, ["S", "V"])
    r2 = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, bnf, ["S", "V"])
    for a in ("S", "V"):
        assert np.array_equal(r1[a][1], r2[a][1])
        bits = np.unpackbits(r1[a][1].view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
        assert np.array_equal(bits, bits.T)
    assert r1["S"][0] > 0


def test_rpq_rows_match_all_pairs_and_threads():
    g = synth.powerlaw(500, seed=11)
    full = oracle.rpq_all(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2)
    srcs = np.array([0, 7, 123, 499, 7], dtype=np.uint32)
    rows = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=4)
    assert np.array_equal(rows, full[srcs])
    r = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, "S -> " + synth.RPQ_C2)
    assert np.array_equal(r["S"][1], full)


def test_plain_definition_not_method_output_monotone():
    # adding edges never removes pairs (the relation is monotone in the graph)
    g = synth.erdos_renyi(64, seed=12)
    r1 = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.BRACKETS)["S"][1]
    extra = synth.erdos_renyi(64, seed=13)
    src = np.concatenate([g.src, extra.src])
    lbl = np.concatenate([g.lbl, extra.lbl])
    dst = np.concatenate([g.dst, extra.dst])
    r2 = oracle.cfl_reach(g.n, src, lbl, dst, g.labels, synth.BRACKETS)["S"][1]
    assert np.array_equal(r1 & r2, r1)
