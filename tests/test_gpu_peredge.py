"""The literal per-edge incremental closure arm (CFPQ_STRATEGY_PEREDGE,
Sec. 3.1.1) against the oracle, and against the frontier-incremental levels
strategy on iterations and per-iteration new edges (Listing 1's Jacobi
order fixes both: they do not depend on how the closure is computed)."""
import json
import os

import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod
from tests import helpers as H

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfpq.load()


def both(g, R):
    graph, q = cfpq.Graph.from_synth(g), cfpq.Query(R)
    pe = cfpq.query(graph, q, strategy=cfpq.STRATEGY_PEREDGE)
    lv = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS)
    return pe, lv


def test_paper_example_iterations_and_deltas():
    fx = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    g = synth.make_graph(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    for R in (rsm_mod.paper_example_rsm(g.labels), rsm_mod.from_grammar(fx["grammar"], g.labels)):
        pe, lv = both(g, R)
        assert {tuple(p) for p in pe.pairs(0).tolist()} == {tuple(p) for p in fx["S"]}
        it, deltas, _ = pe.stats()
        assert it == 3 and deltas == [1, 1, 0]


@pytest.mark.parametrize("k", [1, 3, 6])
def test_chain_closed_form(k):
    g = synth.chain("a" * k + "b" * k)
    pe, _ = both(g, rsm_mod.from_grammar(synth.BRACKETS, g.labels))
    assert {tuple(p) for p in pe.pairs(0).tolist()} == {(k - j, k + j) for j in range(1, k + 1)}
    assert pe.stats()[0] == k + 1


CASES = [
    ("brackets256", lambda: synth.erdos_renyi(256, seed=synth.BASE_SEED + 1), "cfg", synth.BRACKETS),
    ("brackets97", lambda: synth.erdos_renyi(97, seed=synth.BASE_SEED + 801), "cfg", synth.BRACKETS),
    ("samegen", lambda: synth.hierarchy(300, seed=synth.BASE_SEED + 802)[0], "cfg", synth.SAME_GEN_G1),
    ("samegen_g2", lambda: synth.hierarchy(250, seed=synth.BASE_SEED + 803)[0], "cfg", synth.SAME_GEN_G2),
    ("alias", lambda: synth.clustered(300, cluster=(16, 64), seed=synth.BASE_SEED + 804), "cfg", synth.MEM_ALIAS),
    ("nullable", lambda: synth.erdos_renyi(130, seed=synth.BASE_SEED + 805), "cfg", "S -> a S b S | eps"),
    ("rpq", lambda: synth.powerlaw(500, seed=synth.BASE_SEED + 806), "regex", synth.RPQ_C2),
]


@pytest.mark.parametrize("name,make,kind,text", CASES, ids=[c[0] for c in CASES])
def test_matches_oracle_and_levels(name, make, kind, text):
    print(f"peredge: {name}", flush=True)
    g = make()
    R = H.compile_query(kind, text, g.labels)
    pe, lv = both(g, R)
    if kind == "regex":
        want = {R.box_names[0]: H.oracle_regex(g, text)}
    else:
        want = {a: bm for a, (_, bm) in H.oracle_grammar(g, text).items()}
    for b, name_b in enumerate(R.box_names):
        got = pe.bitmap(b)
        assert H.padding_clear(got, g.n)
        assert np.array_equal(got, want[name_b]), name_b
        assert pe.count(b) == H.popcount(want[name_b])
        assert pe.hash(b) == lv.hash(b)
    assert pe.stats()[:2] == lv.stats()[:2]


def test_random_queries_match_oracle():
    rng = np.random.default_rng(23)
    labels = [f"l{i}" for i in range(5)]
    for i in range(8):
        g = synth.serving_graph(int(rng.integers(40, 200)), 900 + i, labels)
        text = synth.random_regex(rng, labels) if i % 2 else synth.random_cfg(rng, labels)
        R = rsm_mod.from_regex(text, labels) if i % 2 else rsm_mod.from_grammar(text, labels)
        want = H.oracle_regex(g, text) if i % 2 else H.oracle_grammar(g, text)["N0"][1]
        pe, lv = both(g, R)
        assert np.array_equal(pe.bitmap(0), want), text
        assert pe.stats()[:2] == lv.stats()[:2]


def test_limits_and_options():
    g = synth.chain("ab" * 9000)      # 18,001 vertices: states * n beyond 65,536
    R = rsm_mod.from_grammar(synth.BRACKETS, g.labels)
    assert R.n_states * g.n > 65536
    graph, q = cfpq.Graph.from_synth(g), cfpq.Query(R)
    with pytest.raises(cfpq.CfpqError) as e:
        cfpq.query(graph, q, strategy=cfpq.STRATEGY_PEREDGE)
    assert e.value.status == cfpq.ERR_LIMIT
    small = synth.erdos_renyi(64, seed=synth.BASE_SEED + 811)
    gs, qs = cfpq.Graph.from_synth(small), cfpq.Query(rsm_mod.from_grammar(synth.BRACKETS, small.labels))
    with pytest.raises(cfpq.CfpqError) as e:
        cfpq.query(gs, qs, strategy=cfpq.STRATEGY_PEREDGE, keep_rank=True)
    assert e.value.status == cfpq.ERR_INVALID
    # masks filter the start box's relation as for every strategy
    mask = np.zeros(64, dtype=bool)
    mask[::3] = True
    a = cfpq.query(gs, qs, strategy=cfpq.STRATEGY_PEREDGE, src_mask=mask)
    b = cfpq.query(gs, qs, strategy=cfpq.STRATEGY_LEVELS, src_mask=mask)
    assert np.array_equal(a.bitmap(0), b.bitmap(0))
