"""Autotuner logic on the CPU: class keys, candidate sets, the choice of the
fastest measured candidate, and the persisted cache.  Query runs are
replaced by a fake timer (the GPU test runs the real ones)."""
import json

import numpy as np

import synth
from paper_2103_14688_amd import cfpq, rsm, tune


class FakeGraph:
    def __init__(self, n, m):
        self.n, self.m = n, m

    def info(self):
        return self.n, 4, self.m


class FakeQuery:
    def __init__(self, R):
        self.rsm = R


def test_features_and_keys():
    R = rsm.from_regex(synth.RPQ_C2, ["a", "b", "c", "d"])
    f = tune.features(FakeGraph(100000, 400000), R)
    assert f == {"n_log2": 16, "deg_class": 2, "states": 2, "boxes": 1, "grammar": False, "nullable": False}
    assert tune.key_of(f) == "n16-d2-q2-b1-rpq"
    G = rsm.from_grammar("S -> a S b S | eps", ["a", "b"])
    g = tune.features(FakeGraph(300, 600), G)
    assert g["grammar"] and g["nullable"] and tune.key_of(g).endswith("cfg-eps")


def test_candidates_cover_strategies_modes_tiles_and_arms():
    R = rsm.from_regex(synth.RPQ_C2, ["a", "b", "c", "d"])
    c = tune.candidates(tune.features(FakeGraph(100000, 400000), R))
    assert {o["strategy"] for o in c} == {cfpq.STRATEGY_CONDENSED, cfpq.STRATEGY_LEVELS}
    G = rsm.from_grammar(synth.SAME_GEN_G1, ["sc", "type", "sc_r", "type_r"])
    c = tune.candidates(tune.features(FakeGraph(200000, 480000), G))
    assert any(o.get("nt_mode") == cfpq.NT_ROWS for o in c)
    assert any(o.get("recompute") for o in c)
    assert any(o.get("tile_words", 0) > 1200 for o in c)
    small = tune.candidates(tune.features(FakeGraph(500, 1000), G))
    assert small[0]["strategy"] == cfpq.STRATEGY_FUSED
    # the literal per-edge arm only where the product graph is small
    B = rsm.from_grammar(synth.BRACKETS, ["a", "b"])
    assert any(o["strategy"] == cfpq.STRATEGY_PEREDGE for o in tune.candidates(tune.features(FakeGraph(300, 600), B)))
    assert not any(o["strategy"] == cfpq.STRATEGY_PEREDGE for o in c)   # same generation at n = 2e5


def test_picks_fastest_and_persists(tmp_path, monkeypatch):
    G = rsm.from_grammar(synth.SAME_GEN_G1, ["sc", "type", "sc_r", "type_r"])
    feat = tune.features(FakeGraph(200000, 480000), G)
    cands = tune.candidates(feat)
    # fake timings: the recompute arm is fastest, one candidate fails
    def fake_time(graph, q, opts, runs):
        if opts.get("tile_words", 0) > 1200:
            raise cfpq.CfpqError(cfpq.ERR_OOM, "no memory")
        return 0.5 if opts.get("recompute") else 1.0 + 0.1 * opts.get("nt_mode", 0)
    monkeypatch.setattr(tune.Tuner, "_time", staticmethod(fake_time))
    path = tmp_path / "tune.json"
    t = tune.Tuner(str(path))
    opts, entry = t.tune(FakeGraph(200000, 480000), FakeQuery(G))
    assert opts.get("recompute") is True
    assert len(entry["measured"]) == len(cands)
    assert any(m["ms"] is None for m in entry["measured"])
    saved = json.loads(path.read_text())
    assert tune.key_of(feat) in saved
    # a new tuner reads the cache and does not measure again
    monkeypatch.setattr(tune.Tuner, "_time", staticmethod(lambda *a: (_ for _ in ()).throw(AssertionError("ran"))))
    t2 = tune.Tuner(str(path))
    opts2, _ = t2.tune(FakeGraph(200000, 480000), FakeQuery(G))
    assert opts2 == opts
    assert np.isfinite(entry["ms"])
