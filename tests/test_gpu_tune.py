"""Autotuner on the GPU: every candidate it measures gives the oracle's
answer, and the tuned query does too (the choice never changes a result)."""
import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm, tune
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfpq.load()


CASES = [
    ("brackets", lambda: synth.erdos_renyi(300, seed=synth.BASE_SEED + 700), "cfg", synth.BRACKETS),
    ("samegen", lambda: synth.hierarchy(3000, seed=synth.BASE_SEED + 701)[0], "cfg", synth.SAME_GEN_G1),
    ("alias", lambda: synth.clustered(2500, seed=synth.BASE_SEED + 702), "cfg", synth.MEM_ALIAS),
    ("rpq", lambda: synth.powerlaw(4100, seed=synth.BASE_SEED + 703), "regex", synth.RPQ_C2),
    ("nullable", lambda: synth.erdos_renyi(2500, seed=synth.BASE_SEED + 704), "cfg", "S -> a S b S | eps"),
]


@pytest.mark.parametrize("name,make,kind,text", CASES, ids=[c[0] for c in CASES])
def test_every_candidate_and_the_choice_match_the_oracle(tmp_path, name, make, kind, text):
    print(f"tune: {name}", flush=True)
    g = make()
    R = H.compile_query(kind, text, g.labels)
    want = H.oracle_regex(g, text) if kind == "regex" else H.oracle_grammar(g, text)[R.box_names[0]][1]
    graph, q = cfpq.Graph.from_synth(g), cfpq.Query(R)
    for opts in tune.candidates(tune.features(graph, R)):
        res = cfpq.query(graph, q, **opts)
        assert np.array_equal(res.bitmap(0), want), opts
    t = tune.Tuner(str(tmp_path / "t.json"))
    opts, entry = t.tune(graph, q)
    assert all(m["ms"] is not None for m in entry["measured"])
    res = t.query(graph, q)
    assert np.array_equal(res.bitmap(0), want)
    # reloaded from disk: same choice
    assert tune.Tuner(str(tmp_path / "t.json")).tune(graph, q)[0] == opts
