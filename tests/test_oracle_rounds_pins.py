"""Pins for the oracle's second evaluator, ``cfl_reach_rounds`` (least
fixpoint of the normal-form grammar as relation equations, semi-naive rounds
over bitsets), and for its pair-set hash helpers.

The rounds evaluator is pinned to things other than itself:
* a naive relational fixpoint written separately in Python (tests/brute.py)
  and brute-force path enumeration, on tiny random graphs and grammars;
* closed forms: a^k b^k chains, same-depth pairs on trees (the same-generation
  query of Sec. 4.2 without type edges), the worked example of Sec. 3.3;
* library special cases: S -> a b as a scipy Boolean product;
* the worklist evaluator (itself pinned in test_oracle_pins.py) on graphs
  large enough for both list-walked and word-OR compositions, and both
  orders of new and old facts.
The hash helpers are pinned to a numpy evaluation of the published
SplitMix64 definition and to explicit enumeration.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests import brute
from tests.helpers import bitmap_hash, splitmix64_np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairs_of(bm, n):
    return set(oracle.bitmap_pairs(bm, n))


def rounds(g, text, names=None, threads=2):
    return oracle.cfl_reach_rounds(g.n, g.src, g.lbl, g.dst, g.labels, text, names, threads=threads)


def test_rounds_paper_example():
    fx = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    g = synth.make_graph(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    r, _ = rounds(g, fx["grammar"])
    assert pairs_of(r["S"][1], g.n) == {tuple(p) for p in fx["S"]}
    assert r["S"][0] == len(fx["S"])


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 40])
def test_rounds_chain_anbn(k):
    g = synth.chain("a" * k + "b" * k)
    r, _ = rounds(g, synth.BRACKETS)
    assert pairs_of(r["S"][1], g.n) == {(k - j, k + j) for j in range(1, k + 1)}


@pytest.mark.parametrize("n,seed", [(600, 0), (3000, 1)])
def test_rounds_same_generation_closed_form(n, seed):
    g, depth = synth.hierarchy(n, with_type=False, seed=seed)
    r, _ = rounds(g, synth.SAME_GEN_G1, threads=4)
    bits = np.unpackbits(r["S"][1].view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    want = (depth[:, None] == depth[None, :]) & (depth[:, None] >= 1)
    assert np.array_equal(bits, want)
    levels = np.bincount(depth)
    assert r["S"][0] == int((levels[1:] ** 2).sum())


def _sparse(g, name):
    i = g.labels.index(name)
    sel = g.lbl == i
    return sp.csr_matrix((np.ones(int(sel.sum()), dtype=np.int64), (g.src[sel], g.dst[sel])), shape=(g.n, g.n))


@pytest.mark.parametrize("p", [0.01, 0.2])
def test_rounds_concatenation_is_boolean_product(p):
    # p = 0.2 makes the right operand dense enough for word-OR composition
    g = synth.erdos_renyi(150, labels=("a", "b"), p=p, seed=3)
    r, _ = rounds(g, "S -> a b")
    prod = (_sparse(g, "a") @ _sparse(g, "b")).toarray() > 0
    bits = np.unpackbits(r["S"][1].view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, prod)


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
def test_rounds_grammar_brute_force(seed):
    rng = np.random.default_rng(5000 + seed)
    labels = ["a", "b", "c"][: int(rng.integers(1, 4))]
    n = int(rng.integers(1, 5))
    edges = _tiny_graph(rng, n, labels, int(rng.integers(0, 8)))
    prods = _random_bnf(rng, labels, int(rng.integers(1, 4)))
    text = brute.bnf_text(prods)
    g = synth.make_graph(n, edges, labels)
    r, _ = rounds(g, text)
    naive = brute.relational_fixpoint(n, edges, prods)
    for a in {p[0] for p in prods}:
        assert pairs_of(r[a][1], n) == naive[a], (text, edges, a)
        assert r[a][0] == len(naive[a])
    start = prods[0][0]
    assert brute.brute_cfl(n, edges, prods, start, 6) <= pairs_of(r[start][1], n)


CASES = [
    ("brackets", lambda: synth.erdos_renyi(256, seed=synth.BASE_SEED + 101), synth.BRACKETS),
    ("g1", lambda: synth.hierarchy(1500, seed=21)[0], synth.SAME_GEN_G1),
    ("g2", lambda: synth.hierarchy(1500, seed=22)[0], synth.SAME_GEN_G2),
    ("alias", lambda: synth.clustered(1200, seed=23), synth.MEM_ALIAS),
    ("rpq", lambda: synth.powerlaw(800, seed=24), "S -> " + synth.RPQ_C2),
    ("nullable", lambda: synth.erdos_renyi(200, seed=25), "S -> a S b S | eps"),
]


@pytest.mark.parametrize("name,make,text", CASES, ids=[c[0] for c in CASES])
def test_rounds_equals_worklist(name, make, text):
    g = make()
    want = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, text)
    got, nr = rounds(g, text, threads=4)
    assert nr >= 2
    for a in want:
        assert got[a][0] == want[a][0]
        assert np.array_equal(got[a][1], want[a][1]), a


def test_rounds_thread_count_does_not_matter():
    g = synth.clustered(900, seed=31)
    a, na = rounds(g, synth.MEM_ALIAS, threads=1)
    b, nb = rounds(g, synth.MEM_ALIAS, threads=7)
    assert na == nb
    for k in a:
        assert np.array_equal(a[k][1], b[k][1])


def test_rounds_random_serving_grammars_match_worklist():
    rng = np.random.default_rng(41)
    labels = [f"l{i}" for i in range(6)]
    g = synth.serving_graph(400, 42, labels)
    for _ in range(8):
        text = synth.random_cfg(rng, labels)
        want = oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, text)
        got, _ = rounds(g, text, threads=3)
        for a in want:
            assert np.array_equal(got[a][1], want[a][1]), (text, a)


# ---------------------------------------------------------------------------
# pair-set hashes
# ---------------------------------------------------------------------------

def test_splitmix64_published_values():
    # first outputs of SplitMix64 seeded with 0 and 1 (the generator's
    # documented sequence: seed 0 -> 0xe220a8397b1dcdaf)
    assert int(splitmix64_np(np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF
    g = synth.make_graph(2, [(0, "a", 0)], ["a"])
    bm = np.zeros((2, 1), dtype=np.uint64)
    bm[0, 0] = 1
    assert oracle.pairs_hash(bm, 2) == (1, 0xE220A8397B1DCDAF)
    assert g.n == 2


def test_pairs_hash_matches_numpy_definition_and_row_ids():
    rng = np.random.default_rng(51)
    n = 300
    bits = rng.random((n, n)) < 0.05
    bm = np.packbits(np.pad(bits, ((0, 0), (0, 20))), axis=1, bitorder="little").view(np.uint64)
    c, h = oracle.pairs_hash(bm, n, threads=3)
    assert c == int(bits.sum())
    assert h == bitmap_hash(bm, n)
    # rows given as a subset with their own vertex ids add up to the whole
    ids = np.arange(n, dtype=np.uint32)
    part = [oracle.pairs_hash(bm[ids[i::3]], n, row_ids=ids[i::3]) for i in range(3)]
    assert sum(p[0] for p in part) == c
    assert sum(p[1] for p in part) % (1 << 64) == h


def test_groups_hash_is_union_of_squares():
    groups = [[5, 9, 2], [0], [7, 1, 3, 11]]
    n = 12
    bm = np.zeros((n, 1), dtype=np.uint64)
    for grp in groups:
        for u in grp:
            for v in grp:
                bm[u, 0] |= np.uint64(1 << v)
    assert oracle.groups_hash(groups, threads=2) == oracle.pairs_hash(bm, n)
