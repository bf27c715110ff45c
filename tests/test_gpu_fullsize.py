"""GPU parity at the workloads' full sizes: the HIP path (through the C ABI)
against counts and order-independent hashes that the oracle alone computed
(tests/golden/fullsize.json, written by tests/golden/make_goldens.py, which
imports nothing from the product package).  All arithmetic is Boolean, so
every comparison is exact: equal pair count and equal sum of
splitmix64((u << 32) | v) over the pairs.

* power-law RPQ n = 100,000, all 100,000 source rows, under every closure
  strategy and three automata for (a|b)* c d* (minimal 2 states, the
  unminimised 5-state Glushkov automaton, a 4-state one given state by state);
* same-generation G1 and G2 on the hierarchy n = 50,000 with type edges, and
  G1 without type edges at n = 200,000 and n = 500,000 (closed form; the
  larger one runs in source tiles and with write-back blocks of 128 words);
* memory alias on the clustered graph n = 20,000 with 64..512-vertex
  clusters, both nonterminals.
"""
import json
import os

import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize.json")


@pytest.fixture(scope="module")
def gold():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfpq.load()
    with open(GOLDEN) as f:
        data = json.load(f)
    yield data
    torch.cuda.synchronize()


def _same(res, box, want):
    got = (res.count(box), f"{res.hash(box):016x}")
    assert got == (want["count"], want["hash"]), f"GPU {got} vs oracle {(want['count'], want['hash'])}"


_graphs = {}


def _graph(key, make):
    if key not in _graphs:
        _graphs.clear()
        g = make()
        _graphs[key] = (g, cfpq.Graph.from_synth(g))
    return _graphs[key]


RPQ_AUTOMATA = ["minimal", "glushkov", "four_state"]


def _rpq_rsm(which, labels):
    if which == "minimal":
        return rsm_mod.from_regex(synth.RPQ_C2, labels)
    if which == "glushkov":
        return rsm_mod.from_regex(synth.RPQ_C2, labels, minimize=False)
    return rsm_mod.from_automaton(*synth.RPQ_C2_FOUR_STATE, labels)


@pytest.mark.parametrize("automaton", RPQ_AUTOMATA)
@pytest.mark.parametrize("strategy", [cfpq.STRATEGY_AUTO, cfpq.STRATEGY_LEVELS])
def test_rpq_powerlaw_all_rows(gold, automaton, strategy):
    print(f"fullsize: rpq n=100000 automaton={automaton} strategy={strategy}", flush=True)
    want = gold["rpq_powerlaw_n100000"]
    g, graph = _graph("rpq", lambda: synth.powerlaw(100000, seed=synth.BASE_SEED + 2))
    R = _rpq_rsm(automaton, g.labels)
    q = cfpq.Query(R)
    res = cfpq.query(graph, q, strategy=strategy)
    _same(res, 0, want)
    assert res.stats()[0] == 2          # one productive iteration (Sec. 3.1.2)
    # repeated on the same handle (the condensed strategy's one-read path)
    again = cfpq.query(graph, q, strategy=strategy)
    _same(again, 0, want)


def test_rpq_powerlaw_row_blocks(gold):
    """Per block of 5,000 sources, through the source mask: locates a
    difference if the whole-answer hash ever disagrees."""
    print("fullsize: rpq n=100000 per source block", flush=True)
    want = gold["rpq_powerlaw_n100000"]
    g, graph = _graph("rpq", lambda: synth.powerlaw(100000, seed=synth.BASE_SEED + 2))
    q = cfpq.Query(rsm_mod.from_regex(synth.RPQ_C2, g.labels))
    for blk in want["blocks"][::4]:
        mask = np.zeros(g.n, dtype=bool)
        mask[blk["first_source"]:blk["first_source"] + want["block_sources"]] = True
        res = cfpq.query(graph, q, src_mask=mask)
        _same(res, 0, blk)


@pytest.mark.parametrize("which", ["g1", "g2"])
def test_samegen_with_type_n50000(gold, which):
    print(f"fullsize: same generation {which} n=50000", flush=True)
    want = gold[f"samegen_{which}_n50000"]
    g, graph = _graph("samegen50k", lambda: synth.hierarchy(50000, seed=synth.BASE_SEED + 3)[0])
    text = synth.SAME_GEN_G1 if which == "g1" else synth.SAME_GEN_G2
    R = rsm_mod.from_grammar(text, g.labels)
    res = cfpq.query(graph, cfpq.Query(R))
    for name, w in want["boxes"].items():
        _same(res, R.box(name), w)


def test_samegen_typefree_closed_form_n200000(gold):
    print("fullsize: same generation G1 without type edges n=200000 (closed form)", flush=True)
    want = gold["samegen_typefree_n200000"]["boxes"]["S"]
    g, graph = _graph("samegen200k",
                      lambda: synth.hierarchy(200000, with_type=False, seed=synth.BASE_SEED + 3)[0])
    R = rsm_mod.from_grammar(synth.SAME_GEN_G1, g.labels)
    res = cfpq.query(graph, cfpq.Query(R))
    _same(res, 0, want)


def test_alias_clustered_n20000(gold):
    print("fullsize: memory alias n=20000", flush=True)
    want = gold["alias_n20000"]
    g, graph = _graph("alias20k", lambda: synth.clustered(20000, seed=synth.BASE_SEED + 4))
    R = rsm_mod.from_grammar(synth.MEM_ALIAS, g.labels)
    res = cfpq.query(graph, cfpq.Query(R))
    for name, w in want["boxes"].items():
        _same(res, R.box(name), w)


def test_samegen_typefree_closed_form_n500000(gold):
    # the largest hierarchy: a 187 GB closure, so the sources go in tiles,
    # and rows of 7,813 words, so the write-back's blocks are 128 words
    import gc
    import torch
    print("fullsize: same generation G1 without type edges n=500000 (closed form)", flush=True)
    want = gold["samegen_typefree_n500000"]["boxes"]["S"]
    _graphs.clear()
    gc.collect()
    torch.cuda.empty_cache()
    g, graph = _graph("samegen500k",
                      lambda: synth.hierarchy(500000, with_type=False, seed=synth.BASE_SEED + 3)[0])
    R = rsm_mod.from_grammar(synth.SAME_GEN_G1, g.labels)
    res = cfpq.query(graph, cfpq.Query(R))
    try:
        _same(res, 0, want)
    finally:
        del res
        _graphs.clear()
        gc.collect()
